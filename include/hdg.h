/*
 * hdg.h -- C ABI of the MI355X DG solver for the acoustic wave equation on
 * vertex-mapped hybrid hexahedral / wedge / pyramidal / tetrahedral meshes.
 *
 * Method: Chan, Wang, Modave, Remacle, Warburton, "GPU-accelerated
 * discontinuous Galerkin methods on hybrid meshes" (arXiv:1507.02557).
 *   - PDE (Section 2.2): (1/kappa) p_t + div u = 0, rho u_t + grad p = 0 with
 *     kappa, rho constant per element; upwind-penalty flux with
 *     tau_p = 1/{rho c}, tau_u = {rho c}.
 *   - Bases and element forms (Section 2.1, Table forms, GL formulation):
 *     GL nodal hexahedra (strong), nodal tetrahedra (strong), LSC-DG modal
 *     wedges (skew-symmetric), semi-nodal pyramids (skew-symmetric,
 *     quadrature-free operators of Section 2.3.4).
 *   - Stable local time steps from the computed trace constants (Section 3.4,
 *     eq. dtK); multi-rate level binning (Section 2.4).
 *
 * Conventions
 *   - Status codes: 0 = success, negative = error (HDG_E*).  No exception
 *     crosses this interface.  hdg_last_error() returns a message for the
 *     most recent failing call on a context.
 *   - Element types: 0 hexahedron, 1 wedge, 2 pyramid, 3 tetrahedron.
 *   - "host" arguments are read during the call and not retained; "device"
 *     arguments are HIP device pointers owned by the caller, read or written
 *     asynchronously on the context's stream (the call returns before the
 *     copy completes).  The context owns all memory it allocates.
 *   - Field layout (structure of arrays): for element type t with K_t elements
 *     and Np(t) dofs per element, each field is a float array [K_t][Np(t)];
 *     elements of a type are numbered in mesh order.
 *   - Dof meaning per type: hex: values at the (N+1)^3 Gauss-Legendre nodes,
 *     node i + (N+1)(j + (N+1)k); tet: values at the equispaced nodes
 *     (i,j,k), i+j+k <= N, k outermost, i fastest; wedge: coefficients of the
 *     orthonormal basis phi_{i,j,k} of Section 2.1.3 divided by sqrt(J),
 *     index j*Ntri + tri(i,k) (tri: i outer, k inner); pyramid: coefficients
 *     of the unit-norm semi-nodal basis of Section 2.1.4, index
 *     off_k + j(k+1) + i.
 */
#ifndef HDG_H
#define HDG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HDG_OK 0
#define HDG_EINVAL (-1)     /* bad argument (order, type, size, pointer)   */
#define HDG_EMESH (-2)      /* invalid mesh: J <= 0, unmatched faces, ...  */
#define HDG_ENOMEM (-3)     /* device allocation failed                    */
#define HDG_EHIP (-4)       /* HIP runtime error                           */
#define HDG_ENONFINITE (-5) /* non-finite value found in the state         */
#define HDG_ESTATE (-6)     /* call not valid in the context's state       */

#define HDG_HEX 0
#define HDG_WEDGE 1
#define HDG_PYR 2
#define HDG_TET 3

#define HDG_BC_FREE_SURFACE 0 /* p = 0 (Section 2.2)          */
#define HDG_BC_RIGID_WALL 1   /* u . n = 0                     */

/* Operand precision of the element-batched operator products on the matrix
 * cores (the tetrahedra's volume and lift products of Section 2.3.2,
 * Algorithm 4, with lattice traces; every other product is FP32):
 *   HDG_PREC_FP32          FP32 operands (16x16x4 MFMA)
 *   HDG_PREC_FP16X2        split FP16 operands x = hi + lo, operators scaled
 *                          by a power of two per matrix group and element data
 *                          per element column, products hi*hi + hi*lo + lo*hi
 *                          accumulated in FP32 (16x16x32 MFMA)
 *   HDG_PREC_FP16X2_K16    the same split on 16x16x16 MFMA
 *   HDG_PREC_BF16X2        split BF16 operands x = hi + lo (about 16
 *                          significant bits), hi*hi + hi*lo + lo*hi in FP32
 *                          (16x16x16 BF16 MFMA)
 *   HDG_PREC_BF16X3        three-piece BF16 split x = hi + mid + lo (about 24
 *                          bits), the six products with piece orders summing
 *                          to at most 2, in FP32 (16x16x16 BF16 MFMA)
 * State, geometry (computed in FP64), fluxes and updates are FP32 in all
 * modes. */
#define HDG_PREC_FP32 0
#define HDG_PREC_FP16X2 1
#define HDG_PREC_FP16X2_K16 2
#define HDG_PREC_BF16X2 3
#define HDG_PREC_BF16X3 4

#define HDG_PATH_AUTO 0      /* lattice traces + matrix-core tetrahedra where the mesh allows */
#define HDG_PATH_GENERIC 1   /* cubature-point traces on every face, vector kernels */

typedef struct hdg_ctx hdg_ctx;

/* Mesh description (all host pointers, copied by hdg_create).
 *   xyz       [3*n_vert]  vertex coordinates (x,y,z interleaved), float64
 *   type      [n_elem]    element types (HDG_HEX..HDG_TET)
 *   verts     [8*n_elem]  vertex ids per element in the reference vertex
 *                         order of its type, unused entries -1:
 *     hex   (r,s,t): (-1,-1,-1) (1,-1,-1) (1,1,-1) (-1,1,-1)
 *                    (-1,-1,1) (1,-1,1) (1,1,1) (-1,1,1)
 *     wedge (triangle in (r,t), extruded in s): (-1,-1,-1) (1,-1,-1)
 *                    (-1,-1,1) (-1,1,-1) (1,1,-1) (-1,1,1)
 *     pyramid: (-1,-1,-1) (1,-1,-1) (1,1,-1) (-1,1,-1) apex (-1,-1,1)
 *     tet:     (-1,-1,-1) (1,-1,-1) (-1,1,-1) (-1,-1,1)
 *   kappa,rho [n_elem]    bulk modulus and density (> 0)
 *   bc                    boundary condition on every boundary face (the
 *                         mirror states of Section 2.2's flux: free surface
 *                         p = 0, rigid wall u . n = 0)
 *   bc_face   [6*n_elem]  optional per element and local face (the face order
 *                         of the element's type: hex (r=-1, r=1, s=-1, s=1,
 *                         t=-1, t=1), wedge (s=-1, s=1, t=-1, r=-1, r+t=0),
 *                         pyramid (base, r=-1, s=-1, r+t=0, s+t=0), tet
 *                         (t=-1, s=-1, r+s+t=-1, r=-1)): -1 uses bc, 0 / 1
 *                         choose the condition of that face when it lies on
 *                         the boundary; may be NULL
 *   n_hanging, hanging    [3*n_hanging] rows (v, a, b): vertex v is the
 *                         midpoint of the edge (a, b) (may be 0 / NULL).
 * 1:4 non-conforming faces (an extension: the paper's meshes are
 * conforming, Section 4.2).  A triangular face matched by no other element
 * whose three edge midpoints are hanging vertices is a coarse face; the four
 * triangles of its midpoint subdivision, (v0, m01, m20), (v1, m12, m01),
 * (v2, m20, m12), (m01, m12, m20), must each be the unmatched face of one
 * element.  On every sub-face the flux of Section 2.2 is applied pointwise
 * between the fine element's trace and the coarse element's trace there;
 * the coarse element's face integral is the sum over its sub-faces.  Both
 * sides must be tetrahedra, and hanging vertices must lie at the midpoints
 * of their edges (relative tolerance 1e-12), else HDG_EMESH.                */
typedef struct hdg_mesh {
  int64_t n_vert;
  const double* xyz;
  int64_t n_elem;
  const int8_t* type;
  const int64_t* verts;
  const double* kappa;
  const double* rho;
  int32_t bc;
  const int8_t* bc_face;
  int64_t n_hanging;
  const int64_t* hanging;
} hdg_mesh;

/* Create a solver context for order N (1 <= N <= 5) on mesh m (Section 2).
 * Builds the reference operators in FP64 on the host, matches faces, and
 * computes the geometric factors in FP64 on the device.  Work is enqueued on
 * hip_stream (a hipStream_t, may be NULL for the null stream); the call
 * synchronises that stream before returning.  precision: one of the
 * HDG_PREC_* codes above (else HDG_EINVAL).
 * Errors: HDG_EINVAL (N out of range, bad type id, NULL pointer, a bc_face
 * entry other than -1, 0, 1), HDG_EMESH (non-positive Jacobian, a face shared
 * by more than two elements, a malformed non-conforming face),
 * HDG_ENOMEM, HDG_EHIP.  On error *out is NULL. */
int hdg_create(hdg_ctx** out, const hdg_mesh* m, int N, int precision, void* hip_stream);

/* Release the context and all device memory it owns.  NULL is accepted. */
void hdg_destroy(hdg_ctx* ctx);

/* Message for the last failing call on ctx (or for the last failed
 * hdg_create in this thread if ctx is NULL). */
const char* hdg_last_error(const hdg_ctx* ctx);

/* Number of elements of type t, dofs per element, and sample points per
 * element used by hdg_project (hex/tet: the nodes; wedge: the volume
 * cubature; pyramid: the projection rule).  Any output may be NULL. */
int hdg_type_info(const hdg_ctx* ctx, int t, int64_t* n_elem, int32_t* np, int32_t* n_sample);

/* Local stable time steps (Section 3.4, eq. dtK):
 *   dtau_K = C / (C_rhokappa^K C_T(N) C_J^K),
 * C_rhokappa^K = max(tau_p,K kappa_K, tau_u,K / rho_K) (maxima over the
 * element's faces; over the four sub-faces for a non-conforming coarse face),
 * C_J^K = max|J^s| max|1/J| (hex, pyramid, tet) or max|J^s/J| (LSC wedge)
 * over cubature points, C_T(N) the computed trace constants of Appendix B.
 * dt_out (host) receives dtau_K for every element in mesh order [n_elem];
 * dt_min_out (host) the minimum.  Either may be NULL.  cfl = C > 0. */
int hdg_dt(hdg_ctx* ctx, double cfl, double* dt_out, double* dt_min_out);

/* Physical sample points of type t: the images under the element's vertex
 * map (Section 2.1, the vertex-mapped elements of each type) of the
 * reference sample points that hdg_type_info counts.  xyz_dev: device,
 * float64 [K_t][n_sample][3], caller-owned, written asynchronously on the
 * context's stream.  Errors: HDG_EINVAL (type absent from the mesh, NULL). */
int hdg_get_points(hdg_ctx* ctx, int t, double* xyz_dev);

/* Set the state of type t from samples of the four fields at the points of
 * hdg_get_points (device, float64, each [K_t][n_sample], caller-owned):
 * interpolation at nodes (hex, tet: nodal bases of Sections 2.1.1-2.1.2);
 * L2 projection with the element's own mass (wedge, Section 2.1.3, LSC-DG
 * mass = I: u_i = sum_q w_q sqrt(J_q) phi_i(q) f_q; pyramid, Section 2.1.4,
 * diagonal mass J(a_i, b_j): u_i = sum_q w_q J_q phi_i(q) f_q / J(a_i, b_j)).
 * The paper does not say how initial data enter; this is the projection its
 * mass matrices define.  Wedges and pyramids use a device work buffer of
 * 4 K_t n_sample doubles that the call allocates and frees (it synchronises
 * the stream).  Errors: HDG_EINVAL, HDG_ENOMEM, HDG_EHIP. */
int hdg_project(hdg_ctx* ctx, int t, const double* p, const double* ux, const double* uy,
                const double* uz);

/* hdg_project without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, result and errors as hdg_project, with
 * the work buffer taken from a fixed device array of the library
 * (HDG_PROJECT_SCRATCH_BYTES per GPU, held until the process ends): elements
 * are projected in chunks of at most HDG_PROJECT_SCRATCH_BYTES /
 * (32 n_sample) at a time, in stream order.  Nothing is allocated or freed
 * and the stream is not synchronised.  Every call on one GPU shares that
 * array: calls that overlap in time on one GPU (different streams or
 * threads) race and must be serialised by the caller.  Errors: HDG_EINVAL
 * (also when one element's 4 n_sample doubles exceed the array), HDG_EHIP. */
#define HDG_PROJECT_SCRATCH_BYTES (16 * 1024 * 1024)
int hdg_project_noalloc(hdg_ctx* ctx, int t, const double* p, const double* ux, const double* uy,
                        const double* uz);

/* Copy the state (which = 0) or the last right-hand side / LSERK residual
 * (which = 1) of type t into / out of caller device buffers, each float
 * [K_t][Np] (the dofs of the type's basis, Section 2.1; meaning per type in
 * the conventions above).  Asynchronous device-to-device copies on the
 * context's stream; nothing is retained.  hdg_set_state invalidates the
 * traces and the multi-rate history (the next step rebuilds the traces and
 * restarts the history) and leaves the time unchanged.  Errors: HDG_EINVAL. */
int hdg_set_state(hdg_ctx* ctx, int t, const float* p, const float* ux, const float* uy,
                  const float* uz);
int hdg_get_field(hdg_ctx* ctx, int which, int t, float* p, float* ux, float* uy, float* uz);

/* Evaluate the semi-discrete right-hand side dU/dt = M^{-1} A U of the
 * current state (Section 2.2 flux, Section 2.3 volume/surface/update
 * kernels, Section 3.1 for the operator A) into the context's rhs buffers
 * (read with hdg_get_field, which = 1).  Asynchronous.  Errors: HDG_EHIP. */
int hdg_rhs(hdg_ctx* ctx);

/* Advance the state by n_steps single-rate LSERK4 steps of size dt (the
 * Carpenter-Kennedy 5-stage, 4th-order, 2N-storage scheme): per stage
 * res = a_s res + dt rhs(U); U = U + b_s res.  One fused kernel per element
 * type and stage.  Asynchronous on the context's stream. */
int hdg_step(hdg_ctx* ctx, double dt, int64_t n_steps);

/* Launch-shape autotuner (Section 4.3.2: the number of elements a work-group
 * processes is tuned per element type and order).  For the hexahedron and
 * wedge block kernels, times `reps` right-hand-side launches (after one
 * untimed launch) of every batch size the kernel is built with, on the
 * context's mesh and state, with HIP events on the context's stream, and keeps
 * the fastest for all later launches of the context (the wedge multi-rate
 * update at N = 4 stays wavefront-batched).  Results agree with untuned
 * launches to FP32 rounding (a batch size can change the order of a
 * kernel's sums).  Overwrites the right-hand-side buffer
 * (hdg_get_field(1)); the state is only read.  epb_out (host, may be NULL):
 * int32[4], the chosen elements per block per type, 0 where the type is
 * absent or its kernel has no batch size to tune.  Synchronises the stream.
 * Errors: HDG_EINVAL (reps outside [1, 1000]), HDG_ESTATE (profiling on),
 * HDG_EHIP. */
int hdg_autotune(hdg_ctx* ctx, int reps, int32_t* epb_out);

/* hdg_step through a HIP graph: two steps (ten stage launches per element
 * type, with the interface kernel) are captured once on the context's stream
 * and the graph is replayed n_steps / 2 times; an odd last step runs as
 * hdg_step.  The graph is kept for later calls with the same dt (and path)
 * and released by hdg_destroy.  Results are bitwise those of hdg_step: the
 * same kernels with the same arguments.  For many small problems batched
 * into one mesh (disjoint union: one launch per type and stage for all of
 * them) it removes the per-launch host cost.  Errors: HDG_EINVAL (dt <= 0,
 * n_steps < 0), HDG_ESTATE (profiling on), HDG_EHIP (capture or launch). */
int hdg_step_graph(hdg_ctx* ctx, double dt, int64_t n_steps);

/* Time-step constants (Section 3.4).  HDG_DT_REFERENCE: the local step of
 * eq. dtK with the reference element's computed C_T(N) (Appendix B, Table
 * computedTrace) times C_J^K.  HDG_DT_ELEMENT: the mapped element's own
 * trace constant, dtau_K = C / (C_rhokappa^K C_T(N, K)), which Section 3.4
 * (Table bounds) shows to be the tighter bound; it never gives a shorter
 * step, since C_T(N, K) <= C_T(N) C_J^K. */
#define HDG_DT_REFERENCE 0
#define HDG_DT_ELEMENT 1

/* Per-element trace-inequality constants C_T(N, K) (Section 3.2; Section 3.4,
 * the "computed C_T(N,K)" row of Table bounds): the largest eigenvalue of
 * M_s,K v = lambda M_K v, with M_K the element's mass matrix of the method and
 * M_s,K = sum over its faces of sum_q w_q J^s_q phi_i(x_q) phi_j(x_q) on the
 * faces' canonical cubature rules (wedges: the LSC basis phi / sqrt(J); a
 * coarse non-conforming face with its own rule, exact for the degree-2N
 * integrand).  Computed on the device in FP64 (Lanczos per element on
 * M^-1/2 M_s M^-1/2, largest Ritz value by Sturm multisection) from the
 * stored FP32 geometric factors (relative accuracy about 1e-7), once per
 * context and cached.  out (host, double [n_elem], mesh order) receives them.
 * Synchronises the stream.  Errors: HDG_EINVAL (NULL), HDG_ENOMEM, HDG_EHIP. */
int hdg_trace_constants(hdg_ctx* ctx, double* out);

/* Select the constants hdg_dt, hdg_mrab_setup and hdg_advance use
 * (HDG_DT_REFERENCE, the default, or HDG_DT_ELEMENT, which computes the
 * per-element constants if needed).  Errors: HDG_EINVAL (NULL, unknown mode),
 * those of hdg_trace_constants. */
int hdg_set_dt_mode(hdg_ctx* ctx, int mode);

/* Multi-rate set-up (Section 2.4).  Levels l = 1 (coarsest) .. L = n_levels
 * (1 <= L <= 8) with dtau_l = 2^(L-l) dtau_min, dtau_min the smallest local
 * step of hdg_dt(cfl).  Each element takes the coarsest level whose step does
 * not exceed its own stable step; then elements move to finer levels until
 * face neighbours differ by at most one level.  Outputs (host, may be NULL):
 * dt_min_out, level_counts_out [n_levels] (elements per level 1..L),
 * level_out [n_elem] (level per element, mesh order). */
int hdg_mrab_setup(hdg_ctx* ctx, int n_levels, double cfl, double* dt_min_out, int64_t* level_counts_out,
                   int8_t* level_out);

/* Advance by n_coarse multi-rate Adams-Bashforth-3 coarse steps (dtau_1 each;
 * Section 2.4).  Per substep of dtau_min, the active levels evaluate their
 * right-hand side (a coarser neighbour in mid-step supplies the AB3 dense
 * output of its step at the half point) and take an AB3 step of their own
 * dtau_l.  The first call after hdg_mrab_setup or a state change runs a
 * start-up of two coarse steps of LSERK4 at dtau_min that fills the history.
 * *t_advanced (host, may be NULL) receives the simulated time advanced.
 * Errors: HDG_ESTATE if hdg_mrab_setup was not called. */
int hdg_mrab_advance(hdg_ctx* ctx, int64_t n_coarse, double* t_advanced);

/* Level census of the multi-rate set-up (Section 2.4), for cost accounting:
 * out (host, int64 [4][L][2], L = n_levels of the last hdg_mrab_setup) receives
 * per element type t and level l = 1..L the number of elements, at
 * out[(t L + l - 1) 2], and the number of those that have a face neighbour
 * (across a sub-face too) on a finer level and so write the mid-step traces
 * that neighbour reads, at out[(t L + l - 1) 2 + 1].  Errors: HDG_EINVAL
 * (NULL), HDG_ESTATE (hdg_mrab_setup not called). */
int hdg_mrab_level_info(const hdg_ctx* ctx, int64_t* out);

/* Energy E = 1/2 sum_K (p^T M p / kappa + rho u^T M u) of the current state
 * (Section 3.1: the quantity eq. sym shows the upwind flux cannot increase),
 * with the element mass matrices of Section 2.1, accumulated in FP64 on the
 * device; E (host) receives it.  Synchronises the stream.  Errors:
 * HDG_EINVAL (NULL), HDG_ENONFINITE (E is NaN or Inf; *E is still set). */
int hdg_energy(hdg_ctx* ctx, double* E);

/* Simulated time of the context's state (host value).  hdg_create sets 0;
 * hdg_step adds n_steps dt, hdg_mrab_advance the time it advances,
 * hdg_advance ends at t_final; hdg_project and hdg_set_state leave it
 * unchanged (set it with hdg_set_time).  Errors: HDG_EINVAL (NULL, t not
 * finite). */
int hdg_get_time(const hdg_ctx* ctx, double* t);
int hdg_set_time(hdg_ctx* ctx, double t);

/* Watchdog: HDG_ENONFINITE if any state value of any type is NaN or Inf,
 * else HDG_OK.  Synchronises the stream.  Errors: HDG_EHIP. */
int hdg_check_finite(hdg_ctx* ctx);

#define HDG_STEPPER_LSERK4 0
#define HDG_STEPPER_MRAB3 1

/* Advance from the current time t to t_final (Section 2.2 poses the problem
 * on a time interval [0, T]).  The step is shortened so that it divides the
 * interval exactly:
 *   HDG_STEPPER_LSERK4: n = ceil((t_final - t) / dtau_min) steps of
 *     dt = (t_final - t) / n, dtau_min = min_K dtau_K(cfl) (Section 3.4,
 *     eq. dtK);
 *   HDG_STEPPER_MRAB3 (after hdg_mrab_setup; cfl is ignored, the levels
 *     keep the set-up's): n coarse steps of the levels' coarse step, all
 *     level steps scaled by the same factor <= 1.  If the scaled steps differ
 *     from those of the history in flight (or no history exists yet) the
 *     history is restarted (start-up of two coarse steps, so n >= 2).
 * Every check_every steps (coarse steps for MRAB3; 0: only at the end) and at
 * the end, the state is checked for NaN/Inf; a non-finite state stops the
 * advance with HDG_ENONFINITE.  steps_done (host, may be NULL) receives the
 * steps taken (LSERK4 steps or coarse steps, start-up included).  On success
 * the time is t_final.  Synchronises the stream at each check.  Errors:
 * HDG_EINVAL (t_final < t, cfl <= 0 for LSERK4, bad stepper), HDG_ESTATE
 * (MRAB3 without hdg_mrab_setup), HDG_ENONFINITE, HDG_EHIP. */
int hdg_advance(hdg_ctx* ctx, double t_final, int stepper, double cfl, int64_t check_every,
                int64_t* steps_done);

/* Checkpoint / resume.  A checkpoint holds the time, the state of every
 * type and, when a multi-rate history is in flight, the right-hand-side
 * history of every level (Section 2.4: each level keeps the right-hand sides
 * of its last three steps), the history slot rotation and the level step; a
 * run continued from hdg_checkpoint_load takes bit-identical steps to the
 * uninterrupted one.  host_buf: host memory of hdg_checkpoint_size bytes,
 * caller-owned (save writes it, load reads it; both synchronise the
 * stream).  Loading into a context needs the same mesh and order, and for a
 * multi-rate checkpoint the same hdg_mrab_setup (checked by level counts and
 * a hash of the level of every element).  Errors: HDG_EINVAL (NULL, size too
 * small, checkpoint of another mesh/order/level set-up), HDG_EHIP. */
int hdg_checkpoint_size(const hdg_ctx* ctx, int64_t* bytes);
int hdg_checkpoint_save(hdg_ctx* ctx, void* host_buf, int64_t bytes);
int hdg_checkpoint_load(hdg_ctx* ctx, const void* host_buf, int64_t bytes);

/* Kernel timing for benchmarking.  While enabled (on != 0), the stepping
 * calls bracket every kernel launch with HIP events on the context's stream.
 * hdg_profile_read synchronises the stream and returns the total kernel time
 * in milliseconds (ms_out[12]) and the number of launches (count_out[12])
 * since the last reset, indexed kind * 4 + element type with kind 0 the
 * stage / right-hand-side kernels, 1 the multi-rate update kernels and 2 the
 * non-conforming interface kernel (under HDG_TET); either may be NULL.
 * Enabling or disabling resets the counters. */
int hdg_profile(hdg_ctx* ctx, int on);
int hdg_profile_read(hdg_ctx* ctx, double* ms_out, int64_t* count_out);

/* Kernel path (both compute the same discrete operator, Section 2.3).
 * HDG_PATH_AUTO (default): where no triangular face joins a wedge to a
 * tetrahedron or pyramid, faces between tetrahedra and pyramids exchange
 * face-lattice traces (the traces there are degree-N polynomials, so the
 * lattice values determine them and the flux on a planar face), and
 * tetrahedra (and, at N = 3..5, pyramids) run on the matrix cores, in
 * single-rate and multi-rate stepping.  Otherwise, or with HDG_PATH_GENERIC,
 * every face exchanges traces at the canonical cubature points.
 * hdg_set_path: path is HDG_PATH_AUTO or HDG_PATH_GENERIC (else
 * HDG_EINVAL); HDG_ESTATE after hdg_mrab_setup; HDG_EINVAL for
 * HDG_PATH_GENERIC on a mesh with non-conforming faces (their coupling uses
 * the lattice traces).  Traces are rebuilt from the
 * state on the next step.  hdg_get_path: requested path and whether lattice
 * traces are in use (1) or not (0); either pointer may be NULL. */
int hdg_set_path(hdg_ctx* ctx, int path);
int hdg_get_path(const hdg_ctx* ctx, int* path_out, int* lattice_out);

#ifdef __cplusplus
}
#endif

#endif /* HDG_H */
