/*
 * fedfem.h - C ABI of the MI355X (gfx950) library for the fast explicit
 * dynamics finite element algorithm (FED-FEM) for transient heat transfer of
 * Zhang & Chauhan (arXiv 1909.03355).
 *
 * The library runs the paper's per-time-step hot path on one GPU:
 *   element thermal loads from precomputed geometry and a temperature-
 *   dependent (isotropic, orthotropic or anisotropic) conductivity (Sec. 3.2,
 *   Eq. 17-20), summed at the nodes without a global stiffness matrix
 *   (Sec. 3.1, Eq. 10-12), convection / radiation / flux surface loads
 *   (Sec. 2, Eq. 4, 5, 7) and the explicit update with a lumped capacity
 *   (Sec. 3.1, Eq. 13-16), plus the pre-computation stage of Sec. 3.5 (i) and
 *   the stability bound of Sec. 3.4.
 *
 * Conventions for every function:
 *   - Return value: FED_OK (0) or a negative fed_status.  The message of the
 *     last error on the calling thread is returned by fed_last_error().
 *     No C++ exception crosses this boundary.
 *   - Host arrays passed in are copied before the call returns; the caller
 *     keeps ownership.  Device arrays are hipMalloc'ed device pointers owned
 *     by the caller unless stated otherwise.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Work is
 *     enqueued asynchronously on it; only functions documented as
 *     synchronising wait for it.
 *   - Node and element numbering is the caller's (0-based) everywhere; the
 *     library's internal (tiled) order never leaks out.
 *   - Temperatures are in degrees Celsius, lengths in metres, SI otherwise.
 */
#ifndef FEDFEM_H
#define FEDFEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FED_OK = 0,
  FED_E_ARG = -1,      /* invalid argument (sizes, indices, null pointers, values) */
  FED_E_MESH = -2,     /* inverted or degenerate element, or unusable topology */
  FED_E_UNSTABLE = -3, /* dt above the stability bound, or the health check fired */
  FED_E_HIP = -4,      /* a HIP runtime call failed */
  FED_E_STATE = -5,    /* call made in the wrong state (e.g. step before set_temperature) */
  FED_E_NOMEM = -6     /* device or host allocation failed */
} fed_status;

enum { FED_TET4 = 4, FED_HEX8 = 8 };

/* Arithmetic of the time stepping.  Pre-computation is always FP64. */
enum {
  FED_FP32C = 0, /* FP32 loads and updates, nodal temperatures kept as a compensated
                    (hi, lo) FP32 pair so that thousands of small increments do not
                    round away */
  FED_FP64 = 1,  /* FP64 throughout */
  FED_FP32 = 2   /* plain FP32 (no compensation), for error comparisons */
};

/* Mesh (Sec. 3.5 (i).1).  conn is structure-of-arrays: conn[a*n_elems + e] is the
 * node of local node a of element e.  Hexahedron local order in natural
 * coordinates (xi, eta, zeta): (---)(+--)(++-)(-+-)(--+)(+-+)(+++)(-++), and it
 * must give a positive Jacobian determinant at the centre.  Tetrahedra may have
 * either orientation. */
typedef struct {
  int32_t elem; /* FED_HEX8 or FED_TET4 */
  int64_t n_nodes, n_elems;
  const double *x, *y, *z; /* host, n_nodes each */
  const int32_t *conn;     /* host, elem * n_elems */
} fed_mesh;

/* Material (Sec. 2, Eq. 1): density rho, heat capacity c(T) = c0 + c1 T and
 * conductivity D(T) = k * (s0 + s1 T) with k the symmetric tensor
 * [xx, yy, zz, xy, yz, xz].  Orthotropic: zero off-diagonals; isotropic: equal
 * diagonals.  The factor of D is evaluated at each node of the element and the
 * nodal values averaged (for this linear law: its value at the element's mean
 * nodal temperature); c is evaluated at the node (Sec. 4.2.2).  Materials may differ in every field (different s0, s1
 * cost 2 values per element and step). */
typedef struct {
  double rho, c0, c1;
  double k[6];
  double s0, s1;
} fed_material;

typedef struct {
  int32_t n_materials;
  const fed_material *materials;   /* host, n_materials */
  const int32_t *elem_material;    /* host, n_elems material ids, or NULL (all 0) */
  const double *elem_k;            /* host, 6 * n_elems per-element k tensor (rows of
                                      length n_elems) replacing the material's, or NULL */
  const double *elem_kscale;       /* host, n_elems positive factors on D, or NULL */
  /* Optional piecewise-linear multiplier tables shared by all materials
   * (temperature-dependent properties given as tables, Sec. 4.2.2): n points
   * (2..16, T strictly increasing, f > 0), linear between points and constant
   * beyond the ends.  With a k table, D_e(T) = k_e * (1/n_e) sum_a fk(T_a): the
   * table is evaluated at each node of the element from the node's temperature
   * and the nodal values are averaged (Sec. 4.2.2); every material must have
   * s0 = 1, s1 = 0; with a c table, c_e(T) = c0_e * fc(T) and every
   * material must have c1 = 0.  n = 0: no table. */
  int32_t n_ktab;
  const double *ktab_T, *ktab_f;   /* host, n_ktab each */
  int32_t n_ctab;
  const double *ctab_T, *ctab_f;   /* host, n_ctab each */
} fed_materials;

/* Boundary conditions (Sec. 2, Eq. 3-7).  Faces are lumped to their nodes with
 * area |f| / face_nodes each.  Heat into a node from face f is
 *   |f|/n_f * ( -h (T - Ta) - sigma eps ((T - Tz)^4 - (Ta - Tz)^4) + q ),
 * sigma = 5.67e-8.  Faces with eps > 0 that share a node must share Ta.
 * Dirichlet nodes hold dir_T from fed_set_temperature on. */
typedef struct {
  int64_t n_dir;
  const int32_t *dir_nodes; /* host */
  const double *dir_T;      /* host */
  int64_t n_faces;
  int32_t face_nodes;       /* 3 (triangle) or 4 (bilinear quad) */
  const int32_t *faces;     /* host, faces[f*face_nodes + b] */
  const double *face_h, *face_Ta, *face_eps, *face_q; /* host, n_faces each; NULL = 0 */
  int64_t n_pt;
  const int32_t *pt_nodes;  /* host, concentrated heat inputs (W) */
  const double *pt_W;
  double Tz;                /* absolute zero in Celsius, normally -273.15 */
} fed_bcs;

typedef struct {
  int32_t prec;              /* FED_FP32C, FED_FP64 or FED_FP32 */
  double dt;                 /* > 0: fixed time step; 0: safety * dt_crit */
  double safety;             /* used when dt == 0 (e.g. 0.9) */
  double T_lo, T_hi;         /* temperature range over which dt_crit is bounded and
                                which the health check watches */
  int32_t allow_unstable;    /* 1: accept dt > dt_crit */
  const int32_t *node_instance; /* host, n_nodes instance ids of a batched mesh of
                                   independent instances (one dt per instance), or NULL */
  int32_t tile_nodes;        /* owned nodes per tile; 0 = default (512; resident: the node
                                count over the number of resident workgroups) */
  int32_t block_threads;     /* threads per tile workgroup, a multiple of 64 in [64, 1024]
                                ([64, 512] when fuse_steps > 1); 0 = default (256;
                                resident: 1024) */
  int32_t fuse_steps;        /* K: steps one kernel launch advances (1..4), each tile carrying
                                K element rings of halo; 0 = default (1).  Results do not
                                depend on K. */
  int32_t resident;          /* 1: resident stepping - one launch runs all the steps of a
                                fed_step call, every tile's workgroup holding its elements
                                and nodes in registers for the whole launch and exchanging
                                only halo temperatures with its neighbours through memory.
                                Needs every tile resident at once (FED_E_MESH at fed_create
                                if the mesh does not fit the GPU's resident workgroups) and
                                K = 1.  The launch is an ordinary one: kernels of other
                                streams that hold CUs for seconds make it report FED_E_HIP
                                (its bounded halo waits give up) rather than hang.  Results
                                are bitwise identical to resident = 0 on the same tiles. */
  int32_t hex_gradient;      /* hexahedra: 0 = gradient at the element centre (Eq. 17, the
                                paper's one-point rule); 1 = uniform gradient (the mean of
                                B over the element, W = V), which reproduces linear fields
                                on distorted hexahedra (the patch test of Sec. 4.1); 27
                                values per element instead of 6 (resident stepping reads
                                them from memory every step); fuse_steps <= 1.  Ignored
                                for tetrahedra. */
  double hourglass;          /* eps >= 0 (0 = off): hourglass control of the uniform-
                                gradient hexahedron (not in the paper; the scalar-field form
                                of Flanagan and Belytschko's orthogonal hourglass control).
                                With h_1..h_4 the hourglass patterns of the nodes' natural
                                signs (eta zeta, zeta xi, xi eta, xi eta zeta), b_a the mean
                                gradients and x_a the nodes, gamma_alpha = (h_alpha -
                                sum_i (h_alpha . x_i) b_i) / 8 vanishes on linear fields and
                                the element adds s_e kappa sum_alpha gamma_alpha
                                gamma_alpha^T to its conductance, kappa = eps (tr D / 3) V
                                sum_a |b_a|^2 (1.5 eps k h on a cube of side h).  Damps the
                                four hourglass modes, keeps the patch test, and enters the
                                stability bound and the adjoint; 40 values per element.
                                Needs hex_gradient = 1 (FED_E_ARG otherwise). */
  /* Device memory.  Every device buffer of the context (the pre-computed arrays of
   * Sec. 3.5 (i), the state, checkpoints and adjoint work arrays, and the
   * temporaries of fed_create) comes from dev_alloc(bytes, alloc_ctx), which
   * returns a device pointer of the current device or NULL when it cannot, and
   * goes back through dev_free(ptr, alloc_ctx) once the library no longer uses
   * it: at fed_destroy, or when a call replaces a buffer (the library
   * synchronises the device before giving a buffer back, as hipFree would).
   * Both are called on the thread that calls the library.  NULL for both:
   * hipMalloc and hipFree.  Giving one without the other is FED_E_ARG; a NULL
   * from dev_alloc makes the call fail with FED_E_HIP (out of memory). */
  void *(*dev_alloc)(size_t bytes, void *alloc_ctx);
  void (*dev_free)(void *ptr, void *alloc_ctx);
  void *alloc_ctx;
  /* In-run health check.  The stability bound (Sec. 3.4, Eq. 29) is derived
   * for temperatures in [T_lo, T_hi]: every step's new temperatures are
   * checked against a window (a value outside it or not finite latches the
   * first such step, reported by the next fed_get_temperature as
   * FED_E_UNSTABLE and by fed_health_get; resident launches compare the
   * extremes of every step with the window every 32 steps and at their end,
   * and report the step of the first check that finds one, at most 31 steps
   * late).  check_window 0: the window is [T_lo - m, T_hi + m] with
   * m the largest margin for which the time step in use stays within the
   * bound over the window (the step takes a safety factor below the bound, so
   * it stays provably stable somewhat beyond the range; m = 0 if the step
   * exceeds the bound, no limit where the bound does not depend on T);
   * re-derived by fed_set_range and fed_set_params.  check_window 1: the window
   * is [T_lo - check_margin, T_hi + check_margin].  With
   * check_every > 0, the step that reaches every multiple of check_every
   * (launches end there; with fed_step_graph and one-step launches, the last
   * step of every replay instead) also takes the energy balance of the
   * explicit update: summed over the nodes, C_k (T_k^{n+1} - T_k^n) / dt - Q_k
   * over the nodes that are not Dirichlet minus the conductive load F_k of the
   * Dirichlet nodes is zero (every element's loads sum to zero); the check
   * records its magnitude over the sum of the terms' magnitudes.  The largest
   * is reported by fed_health_get and, when energy_tol > 0 and it exceeds
   * energy_tol, as FED_E_UNSTABLE.  The check step runs in the one-step kernel
   * (same results, bit for bit), so on resident contexts each check ends a
   * resident launch.  check_window 0 or 1; check_margin >= 0; check_every >= 0
   * (0: no energy checks); energy_tol >= 0 (0: report only). */
  int32_t check_window;
  double check_margin;
  int32_t check_every;
  double energy_tol;
} fed_options;

typedef struct fed_ctx fed_ctx;

/* Sizes and traffic of a context (for reporting). */
typedef struct {
  int64_t n_nodes, n_elems, n_instances;
  int64_t n_tiles, n_elems_expanded, n_halo, n_bnd_nodes;
  int32_t elem, prec, block_threads, lds_bytes, fuse_steps, resident;
  double algorithmic_bytes_per_launch; /* unique bytes one K-step launch must move: every
                                          element's entries and operator, every node's state
                                          and coefficients, every boundary record, once */
  double moved_bytes_per_launch;       /* bytes a launch requests, halo copies included */
  double exchange_bytes_per_step;      /* resident stepping: bytes one step moves through
                                          memory (tagged halo reads and export writes); 0
                                          else */
  int32_t resident_adjoint;            /* 1 if fed_backward runs each checkpoint segment's
                                          adjoint steps in one resident launch */
  int32_t reserved_;
  int64_t device_bytes;                /* device memory the context holds now (from the
                                          dev_alloc hook or hipMalloc) */
  double reread_bytes_per_step;        /* resident stepping: bytes one step reads again
                                          beyond the exchange (the operators of the
                                          uniform-gradient hexahedron that do not stay on
                                          chip, re-read every step); 0 else */
} fed_info;

/*
 * Pre-computation stage (Sec. 3.5 (i)): validates the inputs on the host, builds
 * the tiles, then on the GPU in FP64 computes per element det J, B, G (Eq. 17-19)
 * folded into one symmetric 3x3 operator, the lumped capacity (Eq. 14, 21), the
 * per-node surface coefficients and the stability bound dt_crit (Sec. 3.4, Eq. 29;
 * element-eigenvalue bound).  Synchronises `stream`.  On success *out owns all
 * device memory of the context until fed_destroy.
 * Errors: FED_E_ARG (bad sizes/indices/values), FED_E_MESH (det J <= 0 at a hex
 * centre, zero-volume tet, node incidence too high), FED_E_UNSTABLE (dt > dt_crit
 * without allow_unstable), FED_E_HIP, FED_E_NOMEM.
 */
int fed_create(const fed_mesh *mesh, const fed_materials *mats, const fed_bcs *bcs,
               const fed_options *opt, void *stream, fed_ctx **out);

/* Stability bound of the explicit scheme (Sec. 3.4, Eq. 29: dt_crit = 2 /
 * lambda_max, bounded by the element eigenvalues and the boundary terms over
 * [T_lo, T_hi]) and the time step in use, per instance (n = number of entries
 * the arrays can hold; the count is fed_info.n_instances).  Errors: FED_E_ARG
 * (null ctx, n too small). */
int fed_dt(const fed_ctx *ctx, double *dt_crit, double *dt_used, int64_t n);

int fed_info_get(const fed_ctx *ctx, fed_info *out);

/* Initialisation stage (Sec. 3.5 (ii)): sets T (n_nodes FP64, caller order) and
 * applies the essential condition (Eq. 3).  T is a host pointer if on_device == 0,
 * else a device pointer.  Resets the step counter. */
int fed_set_temperature(fed_ctx *ctx, const double *T, int32_t on_device, void *stream);

/* Time-stepping stage (Sec. 3.5 (iii)): enqueues nsteps explicit steps.  Each
 * kernel launch advances K steps (fewer for the remainder); every step computes
 * every element load, sums the loads per node in ascending element order, adds
 * the surface loads and updates T (Eq. 16), keeping Dirichlet nodes fixed.
 * Asynchronous.  FED_E_STATE before fed_set_temperature. */
int fed_step(fed_ctx *ctx, int64_t nsteps, void *stream);

/* Same as fed_step, but replays a captured HIP graph of about `graph_steps`
 * steps (rounded to an even number of K-step launches; 0 = default) for the bulk
 * of the steps.  The graph is captured on a private stream and launched on
 * `stream`. */
int fed_step_graph(fed_ctx *ctx, int64_t nsteps, int32_t graph_steps, void *stream);

/* Copies the current temperatures (FP64, caller order; FP32C returns hi + lo) to
 * T (host if on_device == 0).  Synchronises `stream` and reports the health
 * check (see fed_options): FED_E_UNSTABLE if a temperature left the window or
 * was not finite after any step since fed_set_temperature (or is now), or if
 * the energy residual exceeded energy_tol; FED_E_HIP if a resident launch had
 * to give up waiting for a neighbouring tile (its results are then invalid).
 * The temperatures are copied in every case. */
int fed_get_temperature(fed_ctx *ctx, double *T, int32_t on_device, void *stream);

/* Health record of the steps since fed_set_temperature (or fed_set_state). */
typedef struct {
  int64_t steps;              /* steps taken */
  int64_t first_bad_step;     /* first step after which a temperature was outside the
                                 window or not finite (resident launches: the first of
                                 their checks, every 32 steps, that found one); -1: none
                                 (fed_set_range clears it) */
  double window_lo, window_hi;  /* the window in use (see fed_options) */
  double energy_residual;     /* largest relative energy residual of the checks (0: none) */
  int64_t energy_step;        /* the step of that check; -1: none */
  int64_t energy_checks;      /* energy checks taken */
} fed_health;

/* Reads the health record (synchronises `stream`). */
int fed_health_get(fed_ctx *ctx, fed_health *out, void *stream);

/* Number of steps taken since fed_set_temperature. */
int fed_steps_taken(const fed_ctx *ctx, int64_t *steps);

/* Exact state save/restore (hi and lo arrays of n_nodes values of the working
 * precision: float for FP32C/FP32, double for FP64; lo is ignored except for
 * FP32C), caller order, host memory.  Synchronises `stream`. */
int fed_get_state(fed_ctx *ctx, void *hi, void *lo, int64_t *step, void *stream);
int fed_set_state(fed_ctx *ctx, const void *hi, const void *lo, int64_t step, void *stream);

/* Checkpointing for the adjoint: with every > 0, the state at step 0 (the one
 * fed_set_temperature sets) and after every `every` steps is kept on the device
 * (2 state vectors each; fed_step breaks its launches at those steps).  0 turns
 * it off and frees the checkpoints (another interval frees them too; the same
 * interval reuses them).  Call before fed_set_temperature. */
int fed_checkpoint_every(fed_ctx *ctx, int64_t every);

/* Kept states for the adjoint (resident contexts with checkpointing on): with
 * on != 0 the forward launches also store every step's state (n_nodes values
 * of the working precision a step, per checkpoint segment, allocated as the
 * steps run: about steps x n_nodes x 4 bytes in FP32C), and fed_backward uses
 * them instead of recomputing each segment from its checkpoint.  The
 * derivatives are bit for bit those of the recomputing backward pass.  States
 * count from fed_set_temperature; a fed_set_state in between, or on = 0,
 * makes fed_backward recompute again.  Call after fed_checkpoint_every and
 * before fed_set_temperature.  Errors: FED_E_STATE (not resident, or
 * checkpointing off). */
int fed_keep_states(fed_ctx *ctx, int32_t on);

/* Replaces per-element conductivity factors (kscale, n_elems, > 0), per-element
 * heat capacities (elem_c, n_elems, > 0; the capacity c0 of each element, for
 * materials with c1 = 0) and per-face convection coefficients (face_h, n_faces,
 * >= 0); NULL leaves a set unchanged.  Re-derives on the GPU the element
 * operators, the lumped capacity and the boundary coefficients (Sec. 3.5 (i))
 * and re-checks the stability bound for the time step in use (FED_E_UNSTABLE
 * if it is exceeded and allow_unstable is off).  Arrays are FP64, caller order,
 * host memory if on_device == 0.  Synchronises `stream`. */
int fed_set_params(fed_ctx *ctx, const double *kscale, const double *elem_c,
                   const double *face_h, int32_t on_device, void *stream);

/* Time-varying boundary conditions (the paper's explicit scheme takes the
 * loads of Eq. 4, 5, 7 at the start of every step; Sec. 1 and 5 name real-time
 * use): replaces the per-face ambient temperatures (face_Ta, n_faces), heat
 * fluxes (face_q, n_faces) and concentrated loads (pt_W, n_pt, W; a source that
 * moves along nodes listed at fed_create) for the steps that follow; NULL
 * leaves a set unchanged.  Re-derives the boundary records on the GPU without
 * allocating; the stability bound does not depend on these values.  Radiating
 * faces that share a node must keep a common Ta.  Arrays are FP64, caller
 * order, host memory (validated, and `stream` synchronised before returning)
 * if on_device == 0, else device memory (not validated; asynchronous on
 * `stream`).  Errors: FED_E_ARG (a set the problem does not have, non-finite
 * values, radiating faces at a node with different Ta), FED_E_HIP. */
int fed_set_bc(fed_ctx *ctx, const double *face_Ta, const double *face_q, const double *pt_W,
               int32_t on_device, void *stream);

/* Point-load schedule (the moving and time-varying sources of the paper's
 * real-time use, Sec. 1 and 5, with the loads taken at the start of every
 * step as in the explicit scheme of Sec. 3.1): W holds n_rows rows of n_pt
 * concentrated loads (FP64, row-major, the order of the point loads given at
 * fed_create); step n, counted from fed_set_temperature (or from the step
 * given to fed_set_state), applies row n mod n_rows in place of the loads of
 * fed_create / fed_set_bc.  The GPU derives every row's boundary-record powers
 * once (n_rows x n_bnd_nodes values of the working precision), so the steps
 * read them by index: a resident launch runs any number of scheduled steps,
 * other contexts launch one step at a time (fuse_steps is not used and
 * fed_step_graph runs as fed_step).  The results equal those of calling
 * fed_set_bc(pt_W = row) before every single step, bit for bit, and
 * fed_backward recomputes its segments with the rows of their steps (a run
 * whose loads changed through fed_set_bc between steps is recomputed with the
 * loads in effect when fed_backward is called).  A later fed_set_bc with
 * face_q re-derives the rows; one with pt_W is refused while a schedule is
 * set.  n_rows = 0 removes the schedule (W may then be NULL).  W is host
 * memory (validated; `stream` synchronised before returning) if on_device ==
 * 0, else device memory (not validated, copied in order on `stream`).
 * Allocates device memory when n_rows changes, after synchronising the
 * device.  Errors: FED_E_ARG (no point loads in the problem, n_rows < 0 or
 * above 2^31 - 1, NULL W, non-finite values), FED_E_NOMEM / FED_E_HIP. */
int fed_set_point_schedule(fed_ctx *ctx, const double *W, int64_t n_rows, int32_t on_device,
                           void *stream);

/* Test hook for the failure path of resident stepping (for tests only):
 * spin_limit bounds every halo wait of the context's later fed_step launches
 * (0 = the default, 2^22 polls), and never_match != 0 makes those waits look
 * for a tag no exchange word carries, so each gives up after spin_limit polls.
 * The launch still ends normally, its results are invalid, and the next
 * fed_get_temperature returns FED_E_HIP.  fed_test_waits(ctx, 0, 0) restores
 * normal waits and fed_set_temperature clears the error.  Errors: FED_E_ARG
 * (spin_limit < 0), FED_E_STATE (not a resident context). */
int fed_test_waits(fed_ctx *ctx, int32_t spin_limit, int32_t never_match);

/* Smallest and largest current temperature (FP64; NaN if any is not finite).
 * The stability bound (Sec. 3.4) is derived for [T_lo, T_hi]; a run whose
 * temperatures leave that range should re-derive it with fed_set_range.
 * Synchronises `stream`.  FED_E_STATE before fed_set_temperature. */
int fed_temperature_range(fed_ctx *ctx, double *tmin, double *tmax, void *stream);

/* Re-derives dt_crit (Sec. 3.4, Eq. 29) for the temperature range [T_lo, T_hi]
 * and re-checks the time step in use against it; the health check window
 * follows the new range and its out-of-window record is cleared.  The time step itself is unchanged.  Errors:
 * FED_E_ARG (bad range, c(T) or D(T) not positive on it), FED_E_UNSTABLE (the
 * time step exceeds the new bound and allow_unstable is off; the new bound
 * and range are kept), FED_E_HIP.  Synchronises `stream`. */
int fed_set_range(fed_ctx *ctx, double T_lo, double T_hi, void *stream);

/* Discrete adjoint of the steps taken since fed_set_temperature (not in the
 * paper; it differentiates the explicit recursion of Sec. 3.1 exactly).  For a
 * loss L with gradient dL_dT with respect to the current temperatures (FP64,
 * n_nodes, caller order), runs the steps in reverse, recomputing each
 * checkpoint segment, and returns dL/dlog k_e (g_logk, n_elems), dL/dc_e (g_c,
 * n_elems), dL/dh_f (g_h, n_faces) and dL/dT0 (n_nodes; zero on Dirichlet
 * nodes); any output may be NULL.  Pointers are host memory if on_device == 0,
 * else device.  Temperature-dependent k and c (laws or tables) and radiation
 * are differentiated through; derivatives are taken at the parameters of the
 * context.  A resident context recomputes each segment in one launch and, for
 * hexahedra with the centre-point operator when the tiles fit
 * (fed_info.resident_adjoint), runs the segment's adjoint steps in one launch
 * too; results are bitwise identical either way.  Requires checkpointing on
 * (FED_E_STATE otherwise); FED_E_MESH if a tile needs more LDS than the
 * adjoint kernel can take; FED_E_HIP also if a resident wait gave up.
 * Synchronises `stream`; the forward state is left unchanged. */
int fed_backward(fed_ctx *ctx, const double *dL_dT, double *g_logk, double *g_c, double *g_h,
                 double *dL_dT0, int32_t on_device, void *stream);

/* For callers that cannot allocate device memory (serving loops and harnesses
 * that forbid allocation while they run): fed_backward with the same arguments
 * and the same results, bit for bit, that allocates nothing.  Its work arrays
 * (the recomputed segment's states unless every segment's states were kept,
 * the multiplier pair, the FP64 derivative sums, 1/dt per node and rho V / n_e
 * per element: about (ckpt_every + 4) x n_nodes x 4 + 28 x n_elems bytes in
 * FP32C) are placed in a static array of FED_NOALLOC_SCRATCH_BYTES (64 MiB) that
 * the library's code object holds on every GPU it runs on until the process
 * ends, instead of the context's own buffers.  Every call on a GPU shares that
 * GPU's array and each call initialises what it reads; calls that overlap on
 * one GPU (from two host threads, or on two streams) race and give wrong
 * derivatives.  Errors: those of fed_backward, and FED_E_ARG when the work
 * arrays exceed the array (the message gives both sizes). */
#define FED_NOALLOC_SCRATCH_BYTES (64u << 20)
int fed_backward_noalloc(fed_ctx *ctx, const double *dL_dT, double *g_logk, double *g_c,
                         double *g_h, double *dL_dT0, int32_t on_device, void *stream);

/* Destroys the context and frees its device memory (synchronises the device). */
void fed_destroy(fed_ctx *ctx);

const char *fed_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* FEDFEM_H */
