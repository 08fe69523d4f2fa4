/*
 * dgd.h -- C-ABI of libdgd, a single-GPU (MI355X, gfx950) discontinuous
 * Galerkin solver for diffusion in the extracellular space of an axon
 * substrate, returning the displacement covariance of the ensemble average
 * propagator.
 *
 * The problem follows the paper "A GPU implementation of the Discontinuous
 * Galerkin method for simulation of diffusion in brain tissue" (arXiv
 * 1907.06191):
 *   - section 2.1, eq. (1)-(5): du/dt = div(k grad u) with k = D in the
 *     extracellular region and zero flux (reflecting) on the axon walls;
 *     on the outer box either zero flux (the default) or u = 0 (eq. (4),
 *     absorbing; dgd_operator_build_outer);
 *   - section 2.2: the substrate is a square holding non-overlapping disks;
 *   - section 3.3: the square is cut into pixels, each split by a diagonal
 *     into two triangles (here the lower-left to upper-right diagonal); a
 *     pixel whose centroid lies strictly inside a disk is removed;
 *   - section 3.1: elementwise polynomial approximation on a nodal Lagrange
 *     basis (eq. (8)), advanced in time by a Runge-Kutta method (here
 *     SSP-RK3); the flux is the symmetric interior penalty flux with
 *     penalty sigma = eta p^2 D / h on every interior face;
 *   - section 4.1: from a pulse at each start point x0 the solution is
 *     carried to each diffusion time Delta and the covariance
 *     Sigma = int (x - x0)(x - x0)^T u dx / int u dx is returned.
 *
 * Conventions.  Lengths in micrometres, times in milliseconds, D in
 * um^2/ms.  All functions return 0 (DGD_OK) or a negative DGD_E* code and
 * set a thread-local message readable with dgd_last_error().  No C++
 * exception crosses this boundary.  A handle is used by one host thread at
 * a time.  Host pointers are read during the call only (inputs are copied);
 * device pointers are allocations on the current HIP device.
 */
#ifndef DGD_H
#define DGD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DGD_OK 0
#define DGD_EINVAL (-1)     /* bad argument (size, order, pointer, list) */
#define DGD_ENOMEM (-2)     /* host or device allocation failed, or workspace too small */
#define DGD_EDEVICE (-3)    /* a HIP runtime call failed */
#define DGD_EUNSTABLE (-4)  /* non-finite value or mass drift beyond tolerance */
#define DGD_ENOTFREE (-5)   /* a start point lies outside the box or in a removed cell */

/* Precision of operator and state.  Moments are always reduced in FP64. */
#define DGD_FP64 0
#define DGD_FP32 1
#define DGD_BF16X3 2        /* FP32 state, P3 stages as BF16 hi/lo split products on matrix cores */

/* Condition on the edges of the square (dgd_operator_build_outer). */
#define DGD_OUTER_REFLECT 0 /* zero flux */
#define DGD_OUTER_ABSORB 1  /* u = 0 outside (eq. (4)) */

typedef struct dgd_mesh dgd_mesh;
typedef struct dgd_op dgd_op;
typedef struct dgd_run dgd_run;
typedef struct dgd_batch dgd_batch;

/* Library version as 10000*major + 100*minor + patch. */
int dgd_version(void);

/* Message of the last failing call on this thread ("" if none). */
const char* dgd_last_error(void);

/*
 * Build the pixel-triangle mesh of [0, L]^2 on an n_cells x n_cells grid
 * (h = L / n_cells) with the disks removed (sections 2.2 and 3.3).
 *   disks: host float64 [n_disks][3] = (cx, cy, r); disks may cross the box
 *          edge; n_disks may be 0 (disks may then be NULL).
 * Elements are ordered by cells in vertical strips of "mesh_strip" columns
 * (see dgd_set_option; default 64), each strip row by row, the lower right
 * triangle T0 of a cell before its upper left triangle T1; dgd_mesh_elements
 * reports the order.  The element table goes to the current HIP device when
 * the first operator is built on the mesh.  *out is owned by the
 * caller and released with dgd_mesh_destroy.
 * Errors: EINVAL (L <= 0, n_cells < 1 or > 16383, n_disks < 0, NULL out),
 * ENOMEM, EDEVICE.
 */
int dgd_mesh_create(double L_um, int32_t n_cells, const double* disks, int32_t n_disks,
                    dgd_mesh** out);

/* Counts for reports: active triangles, interior faces, connected
 * components of the face graph, fraction of removed cells.  Any output
 * pointer may be NULL. */
int dgd_mesh_info(const dgd_mesh* mesh, int64_t* n_active, int64_t* n_faces,
                  int32_t* n_components, double* removed_fraction);

/* Element table on the host: cell column, cell row and orientation (0 = T0,
 * 1 = T1) of every active triangle, in solver order.  Arrays of length
 * n_active; any may be NULL. */
int dgd_mesh_elements(const dgd_mesh* mesh, int32_t* cell_i, int32_t* cell_j, int8_t* orient);

/* Face neighbours on the host: for every active triangle in solver order,
 * the element across its faces 0, 1, 2 (T0: bottom, right, diagonal; T1:
 * top, left, diagonal; section 3.3 pixel split), -1 on a wall (a removed
 * cell: no flux), -2 on the square's edge (no flux, or u = 0 with an
 * absorbing operator, eq. (4)).  nbr_out: int32 [n_active][3]. */
int dgd_mesh_faces(const dgd_mesh* mesh, int32_t* nbr_out);

void dgd_mesh_destroy(dgd_mesh* mesh);

/*
 * Build the SIPG operator of degree p on the mesh (section 3.1 with the
 * interior-penalty flux; section 3.2 for the role of the flux).
 *   p in {1, 2, 3}; D > 0 (um^2/ms); eta > 0 (penalty eta p^2 D / h);
 *   precision: DGD_FP64 or DGD_FP32 (state precision; with DGD_FP32 and a
 *     right-hand-side count that is a multiple of 16, P3 stages may run on
 *     matrix cores: option "p3_mfma", by default only where the autotuner
 *     timed them faster than the FP64 vector kernel), or DGD_BF16X3 (p = 3,
 *     zero-flux walls: FP32 state, every RK3 stage contracts the stacked
 *     element stencil on matrix cores as BF16 hi/lo split products --
 *     operator in three BF16 terms, state differences in two, four
 *     products accumulated in FP32, error below about 2^-16 of each
 *     product, from the state's split only -- with
 *     the FP64 per-element mass correction (section 3.1 remark on p <= 3);
 *     runs need a multiple of 16 right-hand sides (EINVAL otherwise), the
 *     Chebyshev exponential runs its FP64 vector path, and batches refuse
 *     such operators);
 *   dt_max_ms > 0: nominal step = min(0.1 h^2 / (D (p+1)^2), dt_max_ms);
 *   dt_max_ms <= 0: nominal step = min(0.1 h^2 / (D (p+1)^2), 0.9 X / b),
 *     X = 2.5127... the real stability limit of SSP-RK3 and
 *     b = 1.05 lambda, lambda a power-iteration estimate of the largest
 *     eigenvalue of M^-1 A computed on the device.
 * The op keeps a pointer to the mesh, which must outlive it.
 * Errors: EINVAL, ENOMEM, EDEVICE.
 */
int dgd_operator_build(const dgd_mesh* mesh, int32_t p, double D_um2_per_ms, double eta,
                       int32_t precision, double dt_max_ms, dgd_op** out);

/*
 * As dgd_operator_build (which is outer = DGD_OUTER_REFLECT), with the
 * condition on the square's edges chosen by `outer`:
 *   DGD_OUTER_ABSORB: u = 0 on the edges (eq. (4), an absorbing boundary),
 *     imposed weakly by the interior-penalty terms of a face whose outside
 *     value is zero: -int (grad u . n) v - int (grad v . n) u + sigma int u v
 *     on every edge face of an active cell.  Mass leaves through the edges,
 *     so dgd_run_moments checks 0 <= M0 <= 1 (to a tolerance, see there)
 *     instead of M0 = 1.  Stages run on the VALU kernels (no matrix-core
 *     path).  Axon walls keep zero flux.
 * Errors: as dgd_operator_build; EINVAL for another `outer`.
 */
int dgd_operator_build_outer(const dgd_mesh* mesh, int32_t p, double D_um2_per_ms, double eta,
                             int32_t precision, double dt_max_ms, int32_t outer, dgd_op** out);

/*
 * The paper's own formulation (eq. (6)-(7) with the fluxes of section
 * 3.2) on all pixels: q = grad u with the central flux (u- + u+)/2 for u,
 * u_t = div(k q) with the harmonic-mean flux 2 k- k+ / (k- + k+) (q- + q+)/2
 * . n for q, k = D in extracellular cells and k = 0 in axon cells, which
 * stay in the mesh (null work there: u keeps its initial value, zero).
 *   mesh: normally built with no disks (every pixel active); cells it has
 *     removed act as zero-flux walls whose u-flux is the inside value.
 *   disks: host float64 [n_disks][3] (cx, cy, r); a cell is an axon cell
 *     when its centroid lies strictly inside a disk (the removal test of
 *     dgd_mesh_create).  The square's edges: zero flux, u-flux the inside
 *     value.
 *   p, D, precision, dt_max_ms: as dgd_operator_build (no penalty; the
 *     power iteration runs on this operator, whose spectral radius is 4x
 *     (P1) to 14x (P3) smaller than that of the primal form at eta = 10).
 * Each RK stage runs two kernels: the gradient pass (q into the run's
 * workspace, 2 np values per element and start point) and the divergence
 * pass with the stage combine.  Start points must lie in extracellular
 * cells (ENOTFREE).  Runs, dgd_eap_solve, the signal and operator apply
 * take this operator; the exponential and batches reject it (EINVAL).
 * Errors: EINVAL, ENOMEM, EDEVICE.
 */
int dgd_operator_build_mixed(const dgd_mesh* mesh, const double* disks, int32_t n_disks, int32_t p,
                             double D_um2_per_ms, int32_t precision, double dt_max_ms,
                             dgd_op** out);

/* Nominal step in ms and the eigenvalue estimate behind it (0 when the
 * caller fixed dt_max_ms).  Either pointer may be NULL. */
int dgd_operator_dt(const dgd_op* op, double* dt_nom_ms, double* lambda_max_per_ms);

/* Nodes per triangle, node coordinates and precision.
 *   nodes: NULL or host float64 [2][np][2]: for orientation o and node k,
 *          the (x, y) position inside the cell in units of h with the cell's
 *          lower-left corner at (0, 0). */
int dgd_operator_info(const dgd_op* op, int32_t* np, double* nodes, int32_t* precision);

/* Device bytes a solve with n_points start points needs (3 state vectors
 * of n_active * np * n_points values plus reduction scratch). */
int dgd_workspace_size(const dgd_op* op, int32_t n_points, size_t* bytes);

/*
 * y = -M^-1 A x (units 1/ms) on device buffers in the op's precision
 * (double for DGD_FP64, float otherwise), layout [n_active][np][n_rhs]
 * with the right-hand-side index fastest.  x and y must not overlap.
 * Asynchronous on hip_stream (NULL: the null stream).
 * Errors: EINVAL, EDEVICE.
 */
int dgd_operator_apply(dgd_op* op, const void* d_in, void* d_out, int32_t n_rhs, void* hip_stream);

void dgd_operator_destroy(dgd_op* op);

/*
 * A run: the state of n_points solves on one operator (section 4.1: one
 * diffusion problem per start point), held on the device in the layout
 * [n_active][np][n_points].
 *
 * dgd_run_create projects the pulse exp(-|x - x0|^2 / (2 sigma0^2)),
 * restricted to the active triangles, onto the space (L2 projection with
 * an FP64 quadrature) and scales each column to unit mass.
 * sigma0 = 0 gives the projected point mass (the Dirac pulse of section
 * 2.1): on the triangle holding x0 (the T0 of its cell when x0 lies on or
 * below the cell's diagonal, else T1), u = M_K^-1 phi(x0), so that
 * int u v = v(x0) for every v of the space; zero elsewhere; mass 1.
 *   points: host float64 [n_points][2]; each must lie in an active cell
 *           (else ENOTFREE).
 *   sigma0_um: >= 0 and finite (else EINVAL).
 *   d_ws: NULL (the library allocates) or a device buffer of ws_bytes >=
 *         dgd_workspace_size bytes that outlives the run (else ENOMEM).
 *   hip_stream: stream every kernel of the run is launched on; NULL gives
 *         the run a stream of its own (default priority).
 */
int dgd_run_create(dgd_op* op, const double* points, int32_t n_points, double sigma0_um,
                   void* d_ws, size_t ws_bytes, void* hip_stream, dgd_run** out);

/* Advance every column by n_steps SSP-RK3 steps of dt_ms (asynchronous on
 * the run's stream; steps are replayed from captured HIP graphs: the first
 * advance with a given dt captures graphs of graph_steps steps and of every
 * power of two up to it, so any later count with that dt only replays). */
int dgd_run_advance(dgd_run* run, int64_t n_steps, double dt_ms);

/* FP64 moments about each start point, host [n_points][6] =
 * (M0, mx, my, Mxx, Mxy, Myy); n_doubles is the capacity of moments_out
 * (EINVAL below 6 n_points).  Synchronises the run's stream.
 * Returns EUNSTABLE if a moment is not finite or |M0 - 1| > the
 * precision's tolerance (1e-9 FP64, 1e-5 otherwise; with an absorbing box
 * M0 outside [-tol, 1 + tol], tol 1e-6 FP64, 1e-5 otherwise, since the
 * discrete solution's mass may exceed 1 by a discretisation error there);
 * moments_out is filled either way. */
int dgd_run_moments(dgd_run* run, double* moments_out, size_t n_doubles);

/* Sizes of a run's host-side buffers: n_values = n_active * np * n_points
 * state values of value_bytes bytes each (4 FP32, 8 FP64), and n_points.
 * Each output may be NULL. */
int dgd_run_shape(const dgd_run* run, int64_t* n_values, int32_t* n_points,
                  int32_t* value_bytes);

/* Narrow-pulse q-space signal of the propagator of each start point (the
 * propagator of section 1; its Fourier transform is the diffusion-weighted
 * signal named in section 5):
 *   E(q) = int u(x) exp(i q . (x - x0)) dx,
 * q in rad/um (no 2 pi).  q: host float64 [n_q][2]; |q| h <= 4 per wave
 * vector.  signal_out: host float64 [n_points][n_q][2] = (re, im).  Element
 * integrals by a 12 x 12 collapsed Gauss-Legendre rule (exact to rounding
 * for |q| h <= 4), FP64 phases from integer cell indices.  Plain runs only
 * (EINVAL for a batch).  Synchronises the run's stream. */
int dgd_run_signal(dgd_run* run, const double* q, int32_t n_q, double* signal_out);

/* Copy the state to or from the host (checkpoint / resume); host buffer of
 * n_active * np * n_points values of the op's state type (dgd_run_shape),
 * layout [element][node][start point]; bytes is the buffer's size: EINVAL
 * when it is smaller (get) or differs (set).  Synchronous.
 * A checkpoint is the state and the step count: FP32 stores round
 * stochastically with the step count in the salt, so a resumed run repeats
 * the uninterrupted one bit for bit when its step count is restored too. */
int dgd_run_get_state(dgd_run* run, void* host_out, size_t bytes);
int dgd_run_set_state(dgd_run* run, const void* host_in, size_t bytes);
/* Steps taken by the run (since creation or the last set). */
int dgd_run_step_count(const dgd_run* run, int64_t* steps_out);
int dgd_run_set_step_count(dgd_run* run, int64_t steps);

/* The stage kernel and launch shape the run uses: kernel 0 = one element
 * and up to 64 right-hand sides per wave, 1 = several elements per wave
 * (at most 32 right-hand sides), 2 = P3 on matrix cores (FP32 products),
 * 3 = P3 on matrix cores (BF16 hi/lo split products, DGD_BF16X3); shape_out
 * (nullable) [4] = (elements per wave, waves per workgroup, XCD band order,
 * workgroups launched).  Errors: EINVAL. */
int dgd_run_kernel(const dgd_run* run, int32_t* kernel_out, int64_t* shape_out);

void dgd_run_destroy(dgd_run* run);

/*
 * Whole solve (section 4.1): for every start point, carry the pulse
 * through the strictly increasing list deltas_ms (all > 0) with the
 * nominal step of the op, landing exactly on each Delta_k
 * (n_k = ceil((Delta_k - Delta_{k-1}) / dt_nom - 1e-9) steps of equal size),
 * and report Sigma about the start point.
 *   sigma_out: host float64 [n_points][n_deltas][3] = (xx, xy, yy);
 *   moments_out: NULL or host float64 [n_points][n_deltas][6].
 * Synchronous.  Errors: as dgd_run_create, plus EINVAL for a bad Delta
 * list and EUNSTABLE as dgd_run_moments.
 */
int dgd_eap_solve(dgd_op* op, const double* points, int32_t n_points, double sigma0_um,
                  const double* deltas_ms, int32_t n_deltas, double* sigma_out,
                  double* moments_out, void* d_ws, size_t ws_bytes, void* hip_stream);

/*
 * dgd_eap_solve for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same solve and outputs, with the run's buffers (three
 * state buffers, start points, partial sums, step counter) in a fixed
 * 64 MiB device array of the library instead of a workspace.  Each GPU the
 * library runs on holds its own copy of that array until the process ends;
 * its address is resolved on the first call on a device.  Makes no
 * hipMalloc/hipFree or other allocating call: the stage launch shape is the
 * tuned one if its key is already in the table (else the option default),
 * steps launch eagerly (no graph), and hip_stream is used as given (NULL:
 * the null stream).  The op's device must be current.
 * Limits and errors: as dgd_eap_solve, plus EINVAL for sigma0_um == 0 (the
 * point-mass upload allocates) or another device current, and ENOMEM when
 * the run needs more than 64 MiB (3 E np R state bytes plus about
 * R (16 + 48 E / 64) bytes).  Calls that overlap on one GPU share the
 * array and race: serialise them (one host thread, or one stream).  The
 * array keeps the last call's contents; everything a call reads is written
 * by that call first.
 */
int dgd_eap_solve_noalloc(dgd_op* op, const double* points, int32_t n_points, double sigma0_um,
                          const double* deltas_ms, int32_t n_deltas, double* sigma_out,
                          double* moments_out, void* hip_stream);

/* dgd_eap_solve with the q-space signal (dgd_run_signal) at every Delta:
 *   signal_out: host float64 [n_points][n_deltas][n_q][2];
 *   moments_out: NULL or host float64 [n_points][n_deltas][6] as in
 *   dgd_eap_solve.
 * Errors: as dgd_eap_solve and dgd_run_signal. */
int dgd_eap_solve_signal(dgd_op* op, const double* points, int32_t n_points, double sigma0_um,
                         const double* deltas_ms, int32_t n_deltas, const double* q, int32_t n_q,
                         double* signal_out, double* moments_out, void* d_ws, size_t ws_bytes,
                         void* hip_stream);

/*
 * Whole solve with the exact semi-discrete flow instead of SSP-RK3: for each
 * interval of the Delta list, u <- exp((Delta_k - Delta_{k-1}) L) u by a
 * Chebyshev expansion on the spectrum [-b, 0] of L = -M^-1 A (Tal-Ezer and
 * Kosloff), the series cut where its remaining coefficients sum below
 * 1e-17.  About 9 sqrt(b (Delta_k - Delta_{k-1}) / 2) operator applications
 * per interval instead of (Delta_k - Delta_{k-1}) / dt RK3 steps.  The
 * state is FP64 whatever the op's precision.
 *   lambda_bound: b, which must bound the largest eigenvalue of M^-1 A;
 *                 <= 0 uses 1.05 x the device power-iteration estimate.
 *   n_applies: NULL or the number of operator applications made.
 * Outputs and errors as dgd_eap_solve (the library allocates, null stream
 * of its own).
 */
int dgd_eap_solve_expm(dgd_op* op, const double* points, int32_t n_points, double sigma0_um,
                       const double* deltas_ms, int32_t n_deltas, double lambda_bound,
                       double* sigma_out, double* moments_out, int64_t* n_applies);

/*
 * Batched solve (section 4.1 over many substrates; the paper's timing table
 * runs 37 start points one after another): n_geoms operators, each on its
 * own mesh, with n_points start points each.  The operators must share h,
 * D, eta and precision; they are grouped by p, and each group advances as
 * one run over the concatenated element tables of its geometries (one
 * fused kernel launch per RK stage for the whole group, replayed from HIP
 * graphs), with the smallest nominal step of its members.
 *   points: host float64 [n_geoms][n_points][2].
 *   d_ws: NULL or >= dgd_batch_workspace_size bytes of device memory.
 */
int dgd_batch_workspace_size(dgd_op* const* ops, int32_t n_geoms, int32_t n_points, size_t* bytes);
int dgd_batch_create(dgd_op* const* ops, int32_t n_geoms, const double* points, int32_t n_points,
                     double sigma0_um, void* d_ws, size_t ws_bytes, void* hip_stream,
                     dgd_batch** out);
/* Groups: count, and per group p, number of geometries, step (ms) and active
 * DoF per right-hand side.  Output arrays may be NULL. */
int dgd_batch_groups(const dgd_batch* batch, int32_t* n_groups, int32_t* group_p,
                     int32_t* group_size, double* group_dt, int64_t* group_dof);
/* Advance one group by n_steps SSP-RK3 steps of dt_ms. */
int dgd_batch_advance(dgd_batch* batch, int32_t group, int64_t n_steps, double dt_ms);
/* FP64 moments, host [n_geoms][n_points][6] (n_doubles: capacity, EINVAL
 * below 6 n_geoms n_points); EUNSTABLE as dgd_run_moments. */
int dgd_batch_moments(dgd_batch* batch, double* moments_out, size_t n_doubles);
/* Geometries and start points per geometry of a batch (outputs nullable). */
int dgd_batch_shape(const dgd_batch* batch, int32_t* n_geoms, int32_t* n_points);
void dgd_batch_destroy(dgd_batch* batch);

/* Whole batched solve through the Delta list (landing schedule per group);
 * sigma_out host [n_geoms][n_points][n_deltas][3], moments_out NULL or
 * [n_geoms][n_points][n_deltas][6].  Synchronous. */
int dgd_eap_solve_batch(dgd_op* const* ops, int32_t n_geoms, const double* points,
                        int32_t n_points, double sigma0_um, const double* deltas_ms,
                        int32_t n_deltas, double* sigma_out, double* moments_out, void* d_ws,
                        size_t ws_bytes, void* hip_stream);

/*
 * Occupancy image of a mesh: image_out host uint8 [size][size], row j (y)
 * slow, column i (x) fast; a pixel is 1 when the grid cell holding the
 * pixel centre ((i + 1/2) L / size, (j + 1/2) L / size) is a removed (axon)
 * cell, else 0.  With size = n_cells the image is the removed-cell mask.
 */
int dgd_mesh_occupancy(const dgd_mesh* mesh, int32_t size, uint8_t* image_out);

/*
 * Learned surrogate (no counterpart in the paper): an ensemble of small
 * networks mapping a 64 x 64 occupancy image and log(Delta / 1 ms) to the
 * three unique entries (xx, xy, yy) of Sigma / (2 D Delta).  Each member:
 * 4 x [conv 3x3 zero-pad -> `channels` maps, ReLU, 2x2 average pool],
 * flatten, append log Delta, 3 x [dense `hidden` units, ReLU], dense 3.
 * Training: mean squared error, Adam (beta 0.9 / 0.999, eps 1e-8), FP32,
 * all forward and backward steps in the library's kernels; every reduction
 * has a fixed order, so results are reproducible bit for bit.
 */
typedef struct dgd_surrogate dgd_surrogate;
/* n_members in [1, 64], channels in [1, 32], hidden in [1, 4096]; weights
 * He-uniform from `seed` (member m uses seed + 7919 m), biases zero. */
int dgd_surrogate_create(int32_t n_members, int32_t channels, int32_t hidden, uint64_t seed,
                         dgd_surrogate** out);
int dgd_surrogate_n_params(const dgd_surrogate* s, int64_t* n);
/* Parameters of one member as one float32 vector (layer order conv1.w,
 * conv1.b, .., conv4.b, fc1.w [hidden][16 channels + 1], fc1.b, fc2.w,
 * fc2.b, fc3.w, fc3.b, head.w [3][hidden], head.b). */
int dgd_surrogate_get_params(const dgd_surrogate* s, int32_t member, float* host_out);
int dgd_surrogate_set_params(dgd_surrogate* s, int32_t member, const float* host_in);
/* Loss and gradient of one member on n <= 4096 samples (no update):
 * images uint8 [n][64][64] in {0, 1}, log_deltas [n], targets [n][3]. */
int dgd_surrogate_loss_grad(dgd_surrogate* s, int32_t member, const uint8_t* images,
                            const double* log_deltas, const double* targets, int32_t n,
                            double* loss_out, float* grad_out);
/* `epochs` passes of mini-batch Adam per member over shuffled full batches
 * of `batch` samples (shuffle from shuffle_seed); epoch_loss_out NULL or
 * [n_members][epochs] mean squared error. */
int dgd_surrogate_train(dgd_surrogate* s, const uint8_t* images, const double* log_deltas,
                        const double* targets, int32_t n, int32_t epochs, int32_t batch,
                        double lr, uint64_t shuffle_seed, double* epoch_loss_out);
/* Ensemble mean [n][3], spread [n] = max over outputs of (max - min) over
 * members (nullable), fallback [n] = spread > threshold (nullable). */
int dgd_surrogate_predict(dgd_surrogate* s, const uint8_t* images, const double* log_deltas,
                          int32_t n, double threshold, double* mean_out, double* spread_out,
                          uint8_t* fallback_out);
void dgd_surrogate_destroy(dgd_surrogate* s);

/* Runtime options (process-wide; read when a run is created or advanced):
 *   "graphs"       1 = replay steps from captured HIP graphs, 0 = plain launches
 *   "graph_steps"  steps of the largest captured graph, 1..4096
 *   "stage_epw"    elements walked by each wave of the stage kernel, 1..256
 *   "stage_waves"  waves per workgroup of the stage kernel, 1..4
 *   "xcd_remap"    1 = each XCD sweeps one contiguous band of elements
 *   "stage_grid"   > 0: persistent stage kernel with this many workgroups
 *   "p3_mfma"      P3 stages with FP32 state on matrix cores
 *                  (v_mfma_f32_16x16x4_f32, FP64 mass correction; the
 *                  right-hand-side count a multiple of 16): 0 = never,
 *                  1 = always, 2 (default) = when the autotuner timed them
 *                  faster than the VALU kernel for the run's key (a
 *                  DGD_BF16X3 operator always runs its split-product kernel)
 *   "mesh_strip"   element order of meshes created afterwards: vertical strips
 *                  of this many cell columns, each row-major (0 = plain rows)
 *   "mesh_group"   element order of meshes created afterwards: the ranked
 *                  cells in runs of this many, each run giving the T0
 *                  triangles of its cells, then their T1 (default 4; 1 = T0,
 *                  T1 per cell), so that aligned runs share an orientation
 *   "packed"       1 (default) = runs with at most 32 right-hand sides use the
 *                  packed stage kernel (4 or 2 elements per wave)
 *   "sort_classes" 1 = packed runs (plain and batched, created afterwards)
 *                  step an element table grouped by class (orientation,
 *                  face mask) within windows of 512 elements and padded per
 *                  class run, so that each wave holds one face mask;
 *                  0 (default) = mesh order.  Host state buffers keep the
 *                  mesh order either way
 *   "autotune"     1 (default) = runs take the tuned stage launch shape of
 *                  their key, tuning it when the run is created if the key
 *                  is new; 0 = the shape options above
 * Errors: EINVAL for an unknown name or a value out of range.
 *
 * Environment: DGD_RUN_LOG = a file to which every dgd_eap_solve,
 * dgd_eap_solve_noalloc and dgd_eap_solve_batch appends one JSON line
 * (configuration, step rule, steps, wall time, update rate, status, mass
 * drift, the start-point mean of Sigma per Delta); DGD_TUNE_CACHE = a file
 * holding the launch-shape table (the text of dgd_tune_export), read before
 * the first lookup and rewritten after every newly tuned key. */
int dgd_set_option(const char* name, int64_t value);

/*
 * Launch-shape autotuner of the stage kernel (the per-stage update of the
 * time loop, section 3.2).  Every launch shape gives the same bits, so the
 * choice only sets the speed.  The search space: elements per wave {1, 2,
 * 4} (1 for the P3 matrix-core kernel), waves per workgroup {1, 2, 4},
 * XCD-banded block order on/off, and a persistent grid of {4, 8, 16}
 * workgroups per compute unit or none.  After a 30 ms warm-up, each shape
 * is timed with HIP events over about 2 ms of launches of the two-input
 * stage (stage input and base state read, output written), twice, in
 * forward and reverse order, and the best four once more; the fastest is
 * stored in a process-wide table under the key
 * (architecture, Np, state precision, kernel, right-hand sides, floor of
 * log2 of the element count).
 *
 * dgd_autotune tunes op at n_points right-hand sides on hip_stream (NULL:
 * the null stream), allocating three state buffers for the trial; shape_out
 * (nullable) [4] = (elements per wave, waves, XCD order, workgroups per CU
 * or 0), ms_out (nullable) = the best time of one stage launch.
 * Synchronous.  Errors: EINVAL, ENOMEM, EDEVICE.
 */
int dgd_autotune(dgd_op* op, int32_t n_points, void* hip_stream, int32_t* shape_out,
                 double* ms_out);
/* The table as text, one line per key: "key epw waves xcd grid_per_cu ms".
 * len_out (nullable) = bytes needed including the terminating NUL; buf may
 * be NULL to query the size, else cap must hold them (EINVAL otherwise). */
int dgd_tune_export(char* buf, size_t cap, size_t* len_out);
/* Merge lines in the export format into the table (EINVAL on a bad line:
 * nothing is merged then).  Lines starting with '#' are skipped. */
int dgd_tune_import(const char* text);
/* Empty the table. */
void dgd_tune_clear(void);

#ifdef __cplusplus
}
#endif

#endif /* DGD_H */
