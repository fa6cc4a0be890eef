/*
 * wdg.h - C ABI of libwdg: reduced-storage nodal DG for first-order acoustics
 * on meshes of vertically mapped wedges, on one AMD MI355X (gfx950).
 *
 * Method: Chan, Wang, Hewett, Warburton, "Reduced storage nodal discontinuous
 * Galerkin methods on semi-structured prismatic meshes" (arXiv:1607.03399).
 *   PDE and fluxes ................ Sec. 2, eq. (form), boundary reflection
 *   nodal wedge basis ............. Sec. 3.1 (triangle Warp & Blend x GLL)
 *   vertically mapped wedges ...... Sec. 3.2, Definition and Lemma 1
 *   Kronecker mass/lift/derivative  Sec. 4.2, triangular lift L^{tri,k}
 *   storage ....................... Sec. 4.3
 *   layered meshes ................ Sec. 5
 *
 * Conventions
 *   - All host pointers are caller-owned, read or written only during the
 *     call and never retained.  Device pointers passed to
 *     wdg_bind_device_state must stay valid while the context uses them.
 *   - Every function returns WDG_OK (0) or a negative WDG_ERR_* code; the
 *     context keeps a message readable with wdg_last_error.  No exception
 *     crosses the ABI and nothing aborts.
 *   - A context is not thread-safe.  Calls follow the state machine
 *     create -> set_mesh -> set_material -> set_fields -> step*; a call made
 *     too early returns WDG_ERR_STATE.
 *   - Elements are numbered as given; wedge nodes are element-major and
 *     within an element n = j * Np_tri + i (j: GLL level from the bottom,
 *     i: triangle node), Np_tri = (N+1)(N+2)/2, Np = Np_tri (N+1).
 *   - Reference domains are bi-unit (triangle r,s >= -1, r+s <= 0;
 *     t in [-1,1]).
 */
#ifndef WDG_H
#define WDG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct wdg_ctx wdg_ctx;

enum {
  WDG_OK = 0,
  WDG_ERR_ARG = -1,           /* bad argument (null pointer, size, range) */
  WDG_ERR_STATE = -2,         /* call out of order for the context state */
  WDG_ERR_NOT_VERTICAL = -3,  /* a wedge violates the vertical-mapping definition (Sec. 3.2) */
  WDG_ERR_JACOBIAN = -4,      /* non-positive Jacobian (zero-volume or inverted element) */
  WDG_ERR_ORIENTATION = -5,   /* bottom triangle not counter-clockwise seen from above */
  WDG_ERR_NONCONFORMING = -6, /* a face is shared by more than two elements */
  WDG_ERR_OUTSIDE = -7,       /* source or receiver point not inside any element */
  WDG_ERR_HIP = -8,           /* HIP runtime error (includes: no device) */
  WDG_ERR_OOM = -9,           /* device allocation failed */
  WDG_ERR_UNSTABLE = -10,     /* non-finite values detected */
  WDG_ERR_UNSUPPORTED = -11   /* not available for this mesh or option */
};

enum { WDG_BC_DIRICHLET_P0 = 0, WDG_BC_RIGID = 1 };
enum { WDG_FLUX_UPWIND = 0, WDG_FLUX_CENTRAL = 1 };
enum { WDG_MASS_EXACT = 0, WDG_MASS_LUMPED = 1 };

/* Create a context for polynomial order 1 <= order_N <= 5 computing in
 * precision_bits = 32 (FP32 fields and operators; FP64 setup) or 64.
 * device >= 0 selects a HIP device; device = -1 creates a host-only context
 * that validates meshes and returns node coordinates but cannot step.
 * Nothing touches the GPU before wdg_set_mesh. */
int wdg_create(int order_N, int precision_bits, int device, wdg_ctx** out);
int wdg_destroy(wdg_ctx* ctx);
/* Message of the last failing call (never NULL; owned by the context). */
const char* wdg_last_error(const wdg_ctx* ctx);

/* Mesh upload (Sec. 3.2, Sec. 5).  vxyz: nv x 3 vertex coordinates.
 * wedge_v: nw x 6 vertex ids; v1,v2,v3 form the bottom triangle,
 * counter-clockwise seen from +z, and v4,v5,v6 lie directly above v1,v2,v3
 * (vertex pairs (1,4),(2,5),(3,6) share x and y to 1e-12 relative to the
 * element size, else WDG_ERR_NOT_VERTICAL).  Every vertical edge must have
 * positive length (WDG_ERR_JACOBIAN).  tet_v: nt x 4 vertex ids of affine
 * tetrahedra with positive orientation (det[v1-v0, v2-v0, v3-v0] > 0, else
 * WDG_ERR_ORIENTATION; degenerate: WDG_ERR_JACOBIAN); nw or nt may be 0.
 * Elements are numbered wedges first, then tetrahedra.  Faces are matched
 * through their vertex ids; unmatched faces are domain boundary.  Tetrahedra
 * meet wedges at triangular faces (Sec. 3.1); a wedge quadrilateral face
 * covered by two tetrahedron triangles (split along one of its diagonals, as
 * when columns of prisms are split into tetrahedra) is coupled on that common
 * refinement; any other partial cover is WDG_ERR_NONCONFORMING.  On
 * success the geometric factors and triangular lifts are built in FP64 (on
 * the device for wedges, on the host for tetrahedra; host-only contexts build
 * host data only).  Material defaults to c = rho = 1, boundary to rigid, flux
 * to upwind, mass to exact, fields to zero. */
int wdg_set_mesh(wdg_ctx* ctx, int64_t nv, const double* vxyz, int64_t nw, const int64_t* wedge_v,
                 int64_t nt, const int64_t* tet_v);

/* Per-element wave speed c > 0 and density rho > 0 (Sec. 2; kappa = rho c^2),
 * arrays of length nw + nt. */
int wdg_set_material(wdg_ctx* ctx, const double* c, const double* rho);
/* Boundary treatment: WDG_BC_DIRICHLET_P0 (p+ = -p-, u+ = u-; Sec. 2) or
 * WDG_BC_RIGID (p+ = p-, u+ = u- - 2 (n.u-) n). */
int wdg_set_boundary(wdg_ctx* ctx, int bc);
/* Numerical flux: WDG_FLUX_UPWIND (tau_p = 1/{rho c}, tau_u = {rho c}; Sec. 2)
 * or WDG_FLUX_CENTRAL (tau = 0; Sec. 4.1). */
int wdg_set_flux(wdg_ctx* ctx, int flux);
/* Wedge mass treatment: WDG_MASS_EXACT (default: exact quadrature with the
 * stored L^{tri,k}, Sec. 4.2-4.3; energy stable) or WDG_MASS_LUMPED
 * (Gauss-Lobatto quadrature in t, Sec. 4.1: block-diagonal mass, not energy
 * stable on vertically varying wedges; kept for comparison).  Applies to
 * the right-hand side and to wdg_energy; tetrahedra are unaffected. */
int wdg_set_mass(wdg_ctx* ctx, int mass);

/* Layer marching (Sec. 7: reuse of the previous layer's data; off by
 * default), on meshes of wedges only, with the level-lane stage kernel
 * (wdg_set_wedge_kernel):
 *   WDG_MARCH_CHUNK: the kernel reads the face nodes of the wedge below or
 *     above from its staged chunk (a run of consecutive layers of one column)
 *     instead of gathering them from memory;
 *   WDG_MARCH_COLUMN: in addition one block marches each column (a run of
 *     consecutive wedges, each the top neighbour of the one before; taller
 *     columns than two chunks of the kernel -- 32 layers at N = 3 in FP32 --
 *     are split into such segments) from the bottom, chunk by chunk, and
 *     keeps a chunk's top level in LDS as the bottom neighbour of the next,
 *     so no triangular face inside a column segment is gathered.
 * Results are bitwise those of WDG_MARCH_OFF with the same kernel.  Other
 * values: WDG_ERR_ARG. */
enum { WDG_MARCH_OFF = 0, WDG_MARCH_CHUNK = 1, WDG_MARCH_COLUMN = 2 };
int wdg_set_layer_march(wdg_ctx* ctx, int mode);

/* Launch shape of the tetrahedron stage kernel (meshes with tetrahedra).
 * The kernel is persistent: each block loads the reference operators once
 * (into registers on the matrix-core variant, into LDS on the vector one) and
 * then loops over chunks of tetrahedra (chunk c, c + blocks, ...).
 * blocks > 0 caps the number of blocks, so that each block runs about
 * chunks / blocks chunks; 0 restores the default cap (the blocks resident on
 * the device at once for the matrix-core variant, 2048 for the vector one).
 * The chunks are independent, so results are bitwise the same for every cap.
 * Negative values: WDG_ERR_ARG. */
int wdg_set_tet_blocks(wdg_ctx* ctx, int blocks);

/* Concurrency of a hybrid stage (meshes with wedges and tetrahedra; Sec. 5).
 * The wedge and tetrahedron kernels of a stage both follow the mortar kernel,
 * read the same stage input and write disjoint nodes.  enable != 0: after the
 * mortar kernel the tetrahedron kernel runs on a second stream of the context
 * (created by wdg_set_mesh, default priority, ordered with the solver stream
 * by events only) while the wedge kernel runs on the solver stream, and the
 * solver stream waits for it before the stage ends; 0 (default): all three
 * kernels in order on the solver stream (side by side the two kernels slow
 * each other down: on the 39 312-wedge + 29 520-tetrahedron N = 4 mesh the
 * step measured 0.83 ms against 0.76 ms in order).  Results are bitwise the
 * same either way.  Stages timed with wdg_kernel_timing always run in order. */
int wdg_set_overlap(wdg_ctx* ctx, int enable);

/* How the tetrahedron stage kernel applies the reference operators D_r, D_s,
 * D_t and LIFT of the affine tetrahedra (Sec. 3.1; standard nodal DG).
 * WDG_TET_MFMA (default): as dense products over a chunk of tetrahedra on the
 * matrix cores (FP32 or FP64 MFMA, per the context precision).
 * WDG_TET_VALU: as per-node dot products on the vector units.  Both compute
 * the same stage up to rounding order.  Other values: WDG_ERR_ARG. */
enum { WDG_TET_MFMA = 0, WDG_TET_VALU = 1 };
int wdg_set_tet_kernel(wdg_ctx* ctx, int variant);

/* Which wedge stage kernel runs (both compute the stage of Sec. 4.2-4.3 up to
 * rounding order).  The level-lane kernel gives each lane one GLL level of an
 * element (the level's triangular slice of the four equations); the
 * node-lane kernel, which exists for orders 4 and 5 in FP32, gives each lane
 * one triangle node (the node's vertical line of GLL levels).  Layer
 * marching and the adjoint sweep always use the level-lane kernel.
 * WDG_WEDGE_AUTO (default): node-lane wherever it exists, else level-lane.
 * WDG_WEDGE_LEVEL: level-lane everywhere.  WDG_WEDGE_NODE: node-lane
 * wherever it exists.  Other values: WDG_ERR_ARG. */
enum { WDG_WEDGE_AUTO = 0, WDG_WEDGE_LEVEL = 1, WDG_WEDGE_NODE = 2 };
int wdg_set_wedge_kernel(wdg_ctx* ctx, int variant);

/* Elements per block of the node-lane wedge kernel (Sec. 6.2: the number of
 * elements a block processes is a tuning parameter).  elements = 0: the
 * built-in default; otherwise one of the compiled shapes, which
 * wdg_batch_trials lists per order (orders 4 and 5 in FP32: 8, 17, 12, 4 and
 * 12, 9, 6, 3, the first of each the default).  Blocks hold whole elements, so
 * results are bitwise the same for every shape.  It applies where the
 * node-lane kernel runs.  Any other value: WDG_ERR_ARG (the setting is kept). */
int wdg_set_wedge_block(wdg_ctx* ctx, int elements);

/* Total number of nodes (sum over elements of Np). */
int wdg_num_nodes(const wdg_ctx* ctx, int64_t* n);
/* Physical node coordinates, num_nodes x 3, in the node order above. */
int wdg_get_node_coords(const wdg_ctx* ctx, double* xyz);

/* Nodal values of p, u_x, u_y, u_z (each num_nodes), e.g. an initial
 * condition by interpolation.  Resets the receiver history. */
int wdg_set_fields(wdg_ctx* ctx, const double* p, const double* ux, const double* uy, const double* uz);
int wdg_get_fields(const wdg_ctx* ctx, double* p, double* ux, double* uy, double* uz);

/* Use caller-owned device memory for the state and a caller-owned HIP stream
 * for every launch.  d_U: 2 * num_nodes * 4 values of the context precision
 * (two ping-pong copies of the node-interleaved state), d_res: num_nodes * 4
 * values; both 256-byte aligned.  Current fields are copied into d_U.  Pass
 * NULL buffers to keep context-owned memory and only set the stream. */
int wdg_bind_device_state(wdg_ctx* ctx, void* d_U, void* d_res, void* hip_stream);

/* Point source s(t) delta(x - xs) in the pressure equation with the Ricker
 * wavelet s(t) = amp (1 - 2 pi^2 f0^2 (t-t0)^2) exp(-pi^2 f0^2 (t-t0)^2).
 * The lowest-numbered element containing xs (1e-12 tolerance in reference
 * coordinates) receives kappa s(t) M^-1 l(xs).  At most 8 sources. */
int wdg_add_ricker_source(wdg_ctx* ctx, const double xyz[3], double f0, double t0, double amp, int* id);
/* Pressure receivers at n points (n x 3), sampled after every completed step;
 * replaces earlier receivers and clears their history. */
int wdg_set_receivers(wdg_ctx* ctx, int64_t n, const double* xyz);
/* Copy the history (steps x n, row = step) into out; *steps receives the
 * number of recorded steps.  out may be NULL to query *steps only. */
int wdg_read_receivers(const wdg_ctx* ctx, double* out, int64_t* steps);

/* Stable time step for a CFL number (reading of Sec. 6: trace inequality):
 * dt = cfl / max_k [ c_k (N+1)(N+3)/3 max_f max J_f / min J ]. */
int wdg_stable_dt(const wdg_ctx* ctx, double cfl, double* dt);
/* Advance nsteps steps of the five-stage fourth-order 2N-storage
 * Runge-Kutta scheme with step dt.  Asynchronous on the bound stream except
 * when receivers are set (their history lives on the device and is read by
 * wdg_read_receivers). */
int wdg_step(wdg_ctx* ctx, int64_t nsteps, double dt);
int wdg_get_time(const wdg_ctx* ctx, double* t);
int wdg_set_time(wdg_ctx* ctx, double t);
/* Wait for all work of the context. */
int wdg_synchronize(wdg_ctx* ctx);

/* Test hook: the semi-discrete right-hand side dU/dt at time t of the state
 * in4 (4 * num_nodes: p block, u_x block, u_y block, u_z block), sources
 * included, written to out4 (same layout).  The context state is unchanged. */
int wdg_eval_rhs(wdg_ctx* ctx, double t, const double* in4, double* out4);
/* wdg_eval_rhs without any device allocation, for callers that cannot
 * allocate (code that must not call hipMalloc: tight serving loops, harnesses
 * that forbid it).  Same arguments, layout and result as wdg_eval_rhs; the
 * state is staged through a 32 MiB device array of the library, which each
 * GPU the library runs on holds until the process ends.  A mesh whose
 * staging does not fit (more nodes than wdg_eval_rhs_noalloc_max_nodes
 * reports for the precision: 524 288 in FP32, 349 525 in FP64) returns
 * WDG_ERR_ARG.  All calls on one GPU share that array: calls that overlap on
 * one GPU (from several host threads) race; each call waits for its stream
 * before returning.  No hipMalloc, hipFree or allocating library call. */
int wdg_eval_rhs_noalloc(wdg_ctx* ctx, double t, const double* in4, double* out4);
/* Largest node count wdg_eval_rhs_noalloc accepts for precision_bits 32 or 64. */
int wdg_eval_rhs_noalloc_max_nodes(int precision_bits, int64_t* n);
/* E = 1/2 sum_k (p^T M^k p / kappa + rho u^T M^k u) (integrand of eq. estab),
 * M^k = M^{tri,k} (x) M^1D (Sec. 4.2), evaluated on the device. */
int wdg_energy(wdg_ctx* ctx, double* E);

/* Gradient of a weighted sum of receiver traces with respect to the
 * per-element wave speed and density, by the discrete adjoint of the whole
 * time-stepped solve.  The forward solve is the one wdg_step runs: nsteps
 * steps of size dt from the current fields and time, with the current sources
 * and material; trace y[n][r] is the pressure at receiver r after step n.
 * With weights w (host, nsteps x nrec, row n = step n) the call returns
 *   grad_c[k] = d/dc_k sum_{n,r} w[n][r] y[n][r],  grad_rho[k] likewise
 * (host arrays of num_elements values); for the misfit
 * 1/2 sum (y - d)^2 pass w = y - d.  The derivative is that of the discrete
 * map (the low-storage Runge-Kutta stages included): the adjoint runs the
 * stage kernels on T E^-1 of the adjoint state, where E is the energy matrix
 * of eq. estab (diag(M^k/kappa, rho M^k)) and T flips the velocity, because
 * the operator is E-skew up to its E-symmetric penalty part (Sec. 2).
 * Forward states are kept every checkpoint_every steps and recomputed
 * segment by segment on the device; device memory used: about
 * nsteps/checkpoint_every + 10 checkpoint_every + 10 states of num_nodes x 4
 * values (nsteps/checkpoint_every + checkpoint_every + 19 under a tight
 * wdg_set_adjoint_memory_limit).  Fields, time and receiver history are unchanged on
 * return.  Meshes of wedges with the exact mass only (tetrahedra, mortars or
 * WDG_MASS_LUMPED: WDG_ERR_UNSUPPORTED); needs receivers (else
 * WDG_ERR_STATE); WDG_ERR_OOM if the buffers do not fit. */
int wdg_adjoint_gradient(wdg_ctx* ctx, int64_t nsteps, double dt, const double* weights, int64_t checkpoint_every,
                         double* grad_c, double* grad_rho);
/* The same gradient for a solve that wdg_step has already run: after
 * wdg_adjoint_record, wdg_step keeps the state at the start of every
 * checkpoint_every-th step (device memory: ceil(max_steps / checkpoint_every)
 * states, kept by the context), so the gradient call skips the forward sweep.
 * The recording covers the steps since the record call; it ends (and
 * wdg_adjoint_gradient_recorded returns WDG_ERR_STATE) when a step of another
 * size runs, max_steps is exceeded, or the fields, time, material, boundary,
 * flux, mass or receivers are set.  weights: recorded steps x nrec (row n:
 * the traces after recorded step n); nsteps (may be NULL) receives the number
 * of recorded steps.  Fields and time are unchanged by the gradient call.
 * While recording, step n's time is t_record + n dt (as the gradient call
 * recomputes it), whatever the split of the steps over wdg_step calls.  When
 * the reverse sweep's buffers are already kept whole-segment (an earlier
 * gradient call with the same checkpoint_every, see
 * wdg_set_adjoint_memory_limit), the recorded steps write their stage inputs
 * and residuals into them, the same bytes as a plain step, and the next
 * gradient call takes its last segment from there instead of recomputing it;
 * a second gradient call of one recording recomputes everything.  Results are
 * identical either way. */
int wdg_adjoint_record(wdg_ctx* ctx, int64_t checkpoint_every, int64_t max_steps);
int wdg_adjoint_gradient_recorded(wdg_ctx* ctx, const double* weights, double* grad_c, double* grad_rho,
                                  int64_t* nsteps);
/* Device-memory budget of the reverse sweep in bytes (0, the default: 85% of
 * the free memory at the call).  Within budget the forward recomputation of
 * a checkpoint segment keeps all its stage data (10 states per step); else it
 * keeps the step-start states and every step recomputes its stages (one more
 * forward pass).  Both give identical results.  The sweep's state buffers
 * stay allocated in the context for later gradient calls (reallocating tens
 * of GB per call can cost more than the sweep); this call and wdg_destroy
 * release them. */
int wdg_set_adjoint_memory_limit(wdg_ctx* ctx, int64_t bytes);

/* Batches: many independent problems (each a context with a wedge mesh of
 * any order, its own material, sources, fields and time step) advanced
 * together.  Each Runge-Kutta stage is one launch per polynomial order over
 * a list of work items (problem, element chunk); one step
 * is captured once as a HIP graph (five stages: a small kernel that writes
 * every problem's stage record on the device -- buffers, coefficients,
 * source amplitudes at the problem's own time -- then the per-order
 * launches, which run concurrently on one stream per order; then a step
 * counter) and replayed.  Each stage launch covers all problems of one order:
 * one block per element chunk of any problem.
 *   wdg_batch_create: device and state precision (32 or 64) of the batch.
 *   wdg_batch_add: a context on that device and precision, with fields set,
 *     meshes of wedges only (else WDG_ERR_UNSUPPORTED); the batch keeps the
 *     pointer (the caller keeps ownership and must not destroy or step the
 *     context while a batch call runs).  index (may be NULL) receives its slot.
 *   wdg_batch_prepare: groups the problems by order and lists their element
 *     chunks problem by problem (one block per chunk, each XCD a contiguous
 *     range); with autotune != 0 (the tuning of elements per block of
 *     Sec. 6.3) times, for every order, the shapes of the stage kernel that
 *     order's problems use alone (wdg_set_wedge_kernel; the node-lane kernel
 *     only if all of them use it) -- the node-lane kernel at four element
 *     counts per block, or the level-lane kernel compiled for 2 waves per
 *     SIMD (as the single-problem kernel) and for 1 (twice the registers) --
 *     on the real data, as the median of five
 *     launches that rewrite only the residual (which the next stage
 *     overwrites anyway), and keeps the fastest; without autotuning the first
 *     candidate (the single-problem kernel's shape).  Then it captures the
 *     step graph.  No problem may be added afterwards (WDG_ERR_STATE).
 *   wdg_batch_step: nsteps steps of every problem from its current fields and
 *     time (each with its own time step); afterwards wdg_get_fields and
 *     wdg_get_time of each context show the new state.  Receiver traces are
 *     not recorded by batch steps, and a forward recording (wdg_adjoint_record)
 *     of a problem ends.
 *   wdg_batch_config: elements per block, the chosen waves per SIMD of order N
 *     and the tuned median stage time of that order (microseconds).
 *   wdg_batch_trials: the autotuner's candidates for order N in the order
 *     tried: kernel (WDG_WEDGE_LEVEL or WDG_WEDGE_NODE), elements per block,
 *     waves per SIMD and median stage time (microseconds); up to cap of them
 *     are written (any array may be NULL), *count receives their number (0
 *     without autotuning).
 * Results are identical to wdg_step of each problem alone. */
typedef struct wdg_batch wdg_batch;
int wdg_batch_create(int device, int precision_bits, wdg_batch** out);
int wdg_batch_destroy(wdg_batch* batch);
const char* wdg_batch_last_error(const wdg_batch* batch);
int wdg_batch_add(wdg_batch* batch, wdg_ctx* problem, double dt, int* index);
int wdg_batch_prepare(wdg_batch* batch, int autotune);
int wdg_batch_step(wdg_batch* batch, int64_t nsteps);
/* How a batch step runs the orders of one stage (performance only; results
 * are identical): enable != 0 (the default) launches each order on its own
 * stream, all at once; 0 launches them one after another on the batch's
 * stream.  Takes effect at the next wdg_batch_step (the step graph is
 * captured again). */
int wdg_batch_set_concurrent(wdg_batch* batch, int enable);
int wdg_batch_config(const wdg_batch* batch, int N, int* elems_per_block, int* waves_per_simd, double* tuned_us);
int wdg_batch_trials(const wdg_batch* batch, int N, int64_t cap, int* kernel, int* elems_per_block,
                     int* waves_per_simd, double* stage_us, int64_t* count);

/* Per-launch timing of the stage kernels with HIP events on the context stream:
 * enable = 1 starts collecting (and clears), 0 stops.  read returns the summed
 * kernel time in milliseconds and the number of timed stages since the last
 * read or enable, waiting for the stream first; the split variant writes
 * ms3[0] wedge kernel, ms3[1] tetrahedron kernel, ms3[2] mortar kernel (a
 * stage runs the mortar kernel of meshes with nonconforming faces, the wedge
 * kernel, then the tetrahedron kernel of hybrid meshes). */
int wdg_kernel_timing(wdg_ctx* ctx, int enable);
int wdg_read_kernel_timing(wdg_ctx* ctx, double* total_ms, int64_t* launches);
int wdg_read_kernel_timing_split(wdg_ctx* ctx, double* ms3, int64_t* launches);

/* Test hook: per-element data built on the device by the FP64 setup kernel,
 * converted to double.  geo: nw x 40 values, slots
 *   0 r_x, 1 r_y, 2 s_x, 3 s_y, 4 t_z J, 5 t_x J (t=-1), 6 t_x J (t=+1),
 *   7 t_y J (t=-1), 8 t_y J (t=+1), 9 kappa, 10 1/rho, 11 rho c,
 *   12..15 bottom face (J_f, n_x, n_y, n_z), 16..19 top face,
 *   20+4e..23+4e quad face on edge e (J_f at its first and second vertex, n_x, n_y),
 *   32..36 rho c of the element plus rho c across each face (bottom, top, quads),
 *   37..39 J_tri h_v / 2, the weights of M^{tri,k} = sum_v (J_tri h_v / 2) M_v
 * (Lemma 1; face Jacobians and normals of Sec. 4.2).  lift: nw x Np_tri x
 * Np_tri, the triangular lift L^{tri,k} = (M^{tri,k})^-1 M^tri (Sec. 4.2),
 * row-major (for N <= 4 the device keeps the lower triangle of
 * (M^{tri,k})^-1 and the product with M^tri is formed here, in FP64).
 * Either pointer may be NULL. */
int wdg_get_element_data(const wdg_ctx* ctx, double* geo, double* lift);

/* Test hook (host only, no device work): the mortar faces of the mesh (a
 * wedge quadrilateral covered by two tetrahedron triangles) and their
 * coupling matrices, integrated on the host in FP64 on the common refinement
 * (Sec. 3.1 and 5; the integrals of the flux on such a face).  Per mortar,
 * faces receives 7 values: wedge, edge e of its quadrilateral, diagonal (0:
 * from the edge's first bottom vertex to the second top vertex, 1: the
 * other), then tetrahedron and face below and above the diagonal (global
 * element ids, wedges first).  couplings receives per mortar and side of the
 * diagonal the lower triangle, packed by columns, of the symmetric
 * n x n matrix int b b^T dA over that side, n = (N+1)^2 + Np_tri, with b the
 * wedge face's Lagrange basis (GLL level m, edge node q, index m (N+1) + q)
 * followed by the tetrahedron face's (face node i): 2 n (n+1)/2 values per
 * mortar.  At most cap mortars are written (either pointer may be NULL);
 * *count receives the number of mortars. */
int wdg_mortar_couplings(const wdg_ctx* ctx, int64_t cap, int64_t* faces, double* couplings, int64_t* count);

/* Host-side reference operators of order N (no context, no device), for
 * inspection.  name: "r","s" (triangle nodes), "t" (GLL nodes), "Dr","Ds"
 * (Np_tri x Np_tri), "Dt","M1" (Nq x Nq), "Mtri", "Mv0","Mv1","Mv2"
 * (Np_tri x Np_tri, int l_a l_b lambda_v), "g0","gN" (Nq), "Ea0".."Ea2",
 * "Eb0".."Eb2" (Np_tri x Nq), "edge0".."edge2" (N+1 node ids); tetrahedron:
 * "tet_r","tet_s","tet_t" (Np_tet nodes), "tet_Dr","tet_Ds","tet_Dt","tet_M"
 * (Np_tet x Np_tet), "tet_LIFT" (Np_tet x 4 Np_tri), "tet_face0".."tet_face3"
 * (Np_tri node ids).  Writes at most cap values; *count receives the full
 * size. */
int wdg_reference_operator(int order_N, const char* name, double* out, int64_t cap, int64_t* count);

#ifdef __cplusplus
}
#endif

#endif /* WDG_H */
