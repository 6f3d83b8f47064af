/*
 * bcm.h -- C ABI of the building-cube projection library for MI355X (gfx950).
 *
 * The library implements the projection part of the paper's fractional-step method
 * (Sec. 3: immersed-body forcing, pressure Poisson equation, velocity correction) on a
 * building-cube mesh (Sec. 2.2: cubes of equal cell count n^3, 2:1 size ratio between
 * face neighbours, a neighbour adjacency table instead of a tree).  The Poisson equation
 * is solved by geometric multigrid coarsened inside each cube (Sec. 3), here wrapped in
 * flexible CG and, in the mixed modes, in FP64 iterative refinement.  On the
 * one-cell-per-cube level the paper runs a conjugate-gradient solve (Sec. 7: at most 10
 * iterations, at most 50 V-cycles); by default this library runs multigrid on the cube graph
 * there instead (coarse_solver), with the paper's CG kept as an option.
 *
 * Conventions shared by every call:
 *   - All field pointers are DEVICE pointers owned by the caller.  Scalar fields are
 *     stored cube-major, [cube][k][j][i] with i fastest, n^3 values per cube, in the
 *     cube order of the mesh description.  Vector fields are passed as three separate
 *     component arrays.
 *   - Field element type: FP64 ("double") in BCM_FP64 and BCM_MIXED; FP32 ("float") for
 *     u, alpha, u_s, u_new, face_u and the velocity cotangents in BCM_MIXED_F32FIELDS.
 *     Pressure, the adjoint pressure and g_p are always FP64.
 *   - The library never allocates device memory: bcm_plan_create reports the workspace
 *     size and the caller binds a buffer of at least that size (bcm_plan_bind).  The first
 *     bind also creates, per plan, a pinned host buffer (136 bytes) for the solver scalars and
 *     one internal stream with two events; bcm_plan_destroy releases them.
 *   - All GPU work is ordered on the caller's stream (a hipStream_t passed as void*;
 *     NULL = the default stream).  On meshes whose cube graph has levels too large for
 *     one workgroup, part of each Krylov iteration runs on the plan's internal stream,
 *     between an event recorded on the caller's stream and one the caller's stream waits
 *     for, so the caller's stream orders it like its own work.
 *     Calls that return solver results wait for the solver's scalars at convergence
 *     checks; the others are asynchronous.
 *   - Return value: BCM_OK (0), a positive warning (outputs valid) or a negative error
 *     (outputs unspecified).  bcm_last_error() returns a thread-local description of the
 *     last error of the calling thread.  No C++ exception crosses this boundary.
 *   - Calls on the same plan must not overlap (they share its workspace).
 */
#ifndef BCM_H
#define BCM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bcm_mesh bcm_mesh;
typedef struct bcm_plan bcm_plan;

enum {
  BCM_OK = 0,
  BCM_NOT_CONVERGED = 1,       /* tolerance not reached within the iteration limits */
  BCM_STAGNATED = 2,           /* tolerance not reached: the true residual stopped decreasing
                                  (an FP64 Krylov pass, or two refinement steps in a row, did
                                  not halve it); the outputs are valid and final_rel_res is
                                  their true residual */
  BCM_ERR_INVALID_ARG = -1,
  BCM_ERR_INVALID_MESH = -2,
  BCM_ERR_WORKSPACE = -3,      /* no workspace bound, or the bound one is too small */
  BCM_ERR_NONFINITE = -4,      /* a residual norm became NaN or Inf */
  BCM_ERR_HIP = -5,            /* a HIP runtime call failed (text in bcm_last_error) */
  BCM_ERR_UNSUPPORTED = -6
};

/* Boundary kind of a cube face on the domain boundary (face_bc). */
enum {
  BCM_BC_NONE = 0,     /* interior face (has a neighbour) */
  BCM_BC_OUTFLOW = 1,  /* open: p = 0 on the face, face velocity = boundary-cell velocity */
  BCM_BC_INFLOW = 2,   /* normal velocity U_in into the domain, dp/dn = 0, never corrected */
  BCM_BC_SLIP = 3      /* zero normal velocity, dp/dn = 0 */
};

/* Precision modes. */
enum {
  BCM_FP64 = 0,             /* everything in FP64 (flexible CG + V-cycle in FP64) */
  BCM_MIXED = 1,            /* FP64 fields, residual and refinement; FP32 sweeps and preconditioner */
  BCM_MIXED_F32FIELDS = 2   /* as BCM_MIXED with FP32 velocity / volume-fraction fields */
};

/*
 * Mesh description (host memory, copied by bcm_mesh_create).  The paper's linear-array
 * mesh (Sec. 2.2): base corner, size (level), cell count and neighbour adjacency.
 *   n          cells per cube edge: 2, 4, 8 or 16
 *   origin     [n_cubes][3] base (minimum) corner of each cube
 *   level      [n_cubes] refinement level, 0 = coarsest; cube edge = root_edge / 2^level
 *   nbr        [n_cubes][6][4] neighbours across faces (-x,+x,-y,+y,-z,+z):
 *                same-level or coarser neighbour: slot 0 = its index, slots 1..3 = -1;
 *                finer neighbours (2:1): the 4 cubes covering the face, slot a + 2b where
 *                a (b) is the lower/upper half along the first (second) tangential axis,
 *                tangential axes in increasing order (x-face: y,z; y-face: x,z; z-face: x,y);
 *                domain boundary: all four slots -1.
 *   face_bc    [n_cubes][6] BCM_BC_* of boundary faces, BCM_BC_NONE on interior faces.
 * Requirements checked by bcm_mesh_create: neighbour links are reciprocal and agree with
 * the geometry, face neighbours differ by at most one level, every boundary face has a
 * kind, and at least one face is BCM_BC_OUTFLOW (so the Poisson problem is nonsingular).
 */
typedef struct {
  int32_t n_cubes;
  int32_t n;
  const double* origin;
  const int8_t* level;
  double root_edge;
  const int32_t* nbr;
  const int8_t* face_bc;
} bcm_mesh_desc;

/* Solver options; bcm_default_opts fills the defaults given in brackets. */
typedef struct {
  int32_t precision;    /* BCM_FP64 / BCM_MIXED / BCM_MIXED_F32FIELDS            [BCM_FP64] */
  double tol;           /* target ||b - A p||_V / ||b||_V, evaluated in FP64       [1e-10] */
  int32_t max_iter;     /* Krylov iterations per solve (FP64 mode) / per inner solve   [50] */
  int32_t max_outer;    /* mixed modes: FP64 refinement steps; FP64 mode: Krylov solves
                           restarted from the true residual (both share max_iter)      [10] */
  double inner_tol;     /* mixed modes: residual reduction asked of each FP32 inner solve
                           (the last one only as much as tol still needs); FP32 rounding
                           of the operator limits what one refinement step gains   [1e-3] */
  int32_t pre_sweeps;   /* red-black Gauss-Seidel sweeps before restriction             [2] */
  int32_t post_sweeps;  /* sweeps after prolongation                                    [2] */
  int32_t coarse_iters; /* CG iterations on the one-cell-per-cube level (coarse_solver 0),
                           or on the smallest cube-graph level when it is not solved
                           directly (coarse_solver 1; at least 64 are used there)      [10] */
  int32_t krylov;       /* 1 = flexible CG preconditioned by one V-cycle, 0 = V-cycles,
                           2 = standard preconditioned CG (one field read fewer per
                           iteration; for preconditioners that do not vary between
                           iterations, so not with coarse_solver 0)                  [1] */
  int32_t coarse_solver;/* one-cell-per-cube level: 0 = CG only (the paper's scheme),
                           1 = multigrid on the cube graph (octree, then lattice merging;
                           box-shaped domains, otherwise 0 is used)                     [1] */
  int32_t coarse_cycles;/* coarse_solver 1: V-cycles per coarse solve                    [1] */
  int32_t graph_split;  /* coarse_solver 1: cube-graph levels with more nodes than this are
                           smoothed by multi-workgroup kernels, the others (and always the
                           smallest) inside one workgroup; -1 = automatic: the leading
                           levels whose x, b and r do not fit in the workgroup's LDS  [-1] */
  int32_t prolong;      /* per-cube multigrid prolongation: 1 = trilinear over the cube's
                           27-neighbourhood (single-level meshes; meshes with 2:1 faces use
                           0), 0 = piecewise constant                                   [1] */
  int32_t check_every;  /* Krylov iterations per convergence check (>= 1).  Each check
                           waits for the solver's scalars on the host; between checks the
                           iterations are enqueued without waiting, so a solve may run up
                           to check_every - 1 iterations past convergence                [1] */
} bcm_solver_opts;

/* Per-call solver report (host memory). */
typedef struct {
  int32_t status;        /* same value as the call's return code */
  int32_t n_outer;       /* refinement steps (mixed) or 1 (FP64) */
  int32_t n_inner;       /* total Krylov (or V-cycle) iterations */
  double final_rel_res;  /* true FP64 relative residual of the returned pressure */
  double* history;       /* caller array of history_cap doubles, or NULL: relative residual
                            at every convergence check (every check_every iterations; inner
                            ones rescaled to the FP64 RHS) */
  int32_t history_cap;
  int32_t history_len;   /* entries written */
} bcm_report;

/* Inputs of one projection step (Sec. 3): u* = (1 - alpha) u~ + alpha u_s; Poisson; correction. */
typedef struct {
  const void* u[3];      /* intermediate velocity u~ (device fields) */
  const void* alpha;     /* solid volume fraction in [0, 1] (device field), NULL = no body */
  const void* us[3];     /* body velocity fields, or all NULL to use us_const */
  double us_const[3];
  double U_in;           /* inflow speed on BCM_BC_INFLOW faces */
  double dt, rho;        /* time step and density (dt/rho scales the correction) */
  const double* p0;      /* initial pressure guess (device, FP64) or NULL (zero) */
} bcm_project_in;

typedef struct {
  void* u_new[3];        /* corrected cell velocity u^{n+1} (device fields) */
  double* p;             /* pressure p^{n+1} (device, FP64, n_cubes * n^3) */
  void* face_u[3];       /* optional corrected face-normal velocities, or NULL each:
                            face_u[d] is [cube][k][j][i] with n+1 entries along axis d
                            (x: [n][n][n+1], y: [n][n+1][n], z: [n+1][n][n]) */
  double* b;             /* optional: the Poisson right-hand side (rho/dt) div U* that was
                            solved (device, FP64), or NULL */
} bcm_project_out;

/* Inputs of the adjoint of one projection step (same forward inputs, no pressure needed:
 * the step is affine in u~ and polynomial in alpha). */
typedef struct {
  const void* u[3];
  const void* alpha;     /* NULL = no body (then g_alpha is not written) */
  const void* us[3];
  double us_const[3];
  double U_in, dt, rho;
  const void* g_u_new[3];  /* cotangent of u^{n+1} (device fields) */
  const double* g_p;       /* cotangent of p^{n+1} (device, FP64) or NULL */
} bcm_adjoint_in;

typedef struct {
  void* g_u[3];          /* cotangent of u~ (written) */
  void* g_alpha;         /* cotangent of alpha (written, or accumulated; ignored when alpha is
                            NULL) */
  double g_U_in;         /* cotangent of U_in (host scalar, written, or accumulated) */
  double* lambda;        /* optional: adjoint pressure A^{-T}(...) (device FP64) or NULL */
  int32_t accumulate;    /* 0: g_alpha and g_U_in are overwritten; 1: this step's cotangents
                            are added to what they hold (the reverse sweep of a multi-step
                            objective sums them over the steps) */
} bcm_adjoint_out;

/* Momentum sub-step schemes (Sec. 3: the paper's code offers Euler, Adams-Bashforth and
 * Crank-Nicolson). */
enum {
  BCM_EULER = 0,  /* u~ = u^n + dt H(u^n) */
  BCM_AB2 = 1,    /* u~ = u^n + dt (3/2 H(u^n) - 1/2 H(u^{n-1})); Euler when h_prev is NULL */
  BCM_CN = 2      /* u~ = u^n + dt/2 (H(u~) + H(u^n)), the advecting velocity frozen at u^n */
};

/* Inputs of the momentum sub-step (Sec. 3, Eq. (substep1)): the intermediate velocity u~ from
 * u^n without body force and pressure, H(v) = -A[v] + nu D[v] with A the QUICK convection in
 * finite-volume flux form (face velocities of u^n: mean of the two cells, as in the projection
 * step) and D the 7-point diffusion; velocity boundary values by two mirrored ghost layers per
 * domain face (inflow: every component fixed, the normal one U_in into the domain; slip: the
 * normal component 0, the tangential ones zero gradient; open: zero gradient). */
typedef struct {
  const void* u[3];       /* u^n (device fields of the field type) */
  const void* h_prev[3];  /* BCM_AB2: H(u^{n-1}) of the previous step (three fields), or all
                             NULL on the first step; ignored by the other schemes */
  double U_in;            /* inflow speed on BCM_BC_INFLOW faces */
  double dt;              /* time step (> 0) */
  double nu;              /* kinematic viscosity mu / rho (>= 0) */
  int32_t scheme;         /* BCM_EULER / BCM_AB2 / BCM_CN */
  double cn_tol;          /* BCM_CN: Jacobi iterations run until ||r||_2 <= cn_tol ||rhs||_2
                             (r = rhs + dt/2 H(x) - x, rhs = u^n + dt/2 H(u^n); 2-norms over
                             all cells and components); 0 = 1e-12 */
  int32_t cn_max_iter;    /* BCM_CN: iteration limit; 0 = 200 */
} bcm_momentum_in;

typedef struct {
  void* u_tilde[3];       /* intermediate velocity u~ (written; must not alias u) */
  void* h[3];             /* optional: H(u^n) (the next AB2 step's h_prev), or all NULL */
} bcm_momentum_out;

/* Surface particles of an immersed body (Sec. 2.3): positions, Lagrangian volumes and the body
 * velocity at each particle. */
typedef struct {
  int32_t n;              /* number of particles (>= 0) */
  const double* X;        /* [n][3] positions (device, FP64) */
  const double* dV;       /* [n] Lagrangian volume dc_1 dc_2 dc_3 of each particle (device), or
                             NULL for h^3 of the cell that holds it */
  const double* Us;       /* [n][3] body velocity at the particles (device), or NULL: us_const */
  double us_const[3];
} bcm_particles;

/* Fill opts with the defaults listed in bcm_solver_opts. */
void bcm_default_opts(bcm_solver_opts* opts);

/* Validate and copy a mesh description (host only, no GPU call).  Errors:
 * BCM_ERR_INVALID_ARG (NULL pointers, bad n), BCM_ERR_INVALID_MESH (the offending cube and
 * face are named in bcm_last_error).  Destroy with bcm_mesh_destroy. */
int bcm_mesh_create(const bcm_mesh_desc* desc, bcm_mesh** out);
void bcm_mesh_destroy(bcm_mesh* mesh);

/* Plan the solver for a mesh and options (host only, no GPU call) and report the device
 * workspace it needs in *workspace_bytes.  The plan keeps a reference to the mesh, which
 * must outlive it. */
int bcm_plan_create(const bcm_mesh* mesh, const bcm_solver_opts* opts, bcm_plan** out,
                    size_t* workspace_bytes);
void bcm_plan_destroy(bcm_plan* plan);

/* Bind a caller-owned device buffer (>= workspace_bytes, 256-byte aligned) to the plan and
 * upload the mesh metadata into it on `stream`.  BCM_ERR_WORKSPACE if too small.  The first
 * bind creates the plan's pinned scalar buffer and internal stream; if either cannot be
 * created the solver copies its scalars back and keeps all work on the caller's stream. */
int bcm_plan_bind(bcm_plan* plan, void* d_workspace, size_t bytes, void* stream);

/* One projection step (Sec. 3, forcing -> Poisson -> correction).  The Poisson solve runs to
 * opts.tol; BCM_NOT_CONVERGED if the limits are hit first and BCM_STAGNATED if the residual
 * stops decreasing first (outputs valid in both cases), BCM_ERR_NONFINITE if a residual norm
 * is not finite.  report may be NULL. */
int bcm_project(bcm_plan* plan, const bcm_project_in* in, bcm_project_out* out,
                bcm_report* report, void* stream);

/* The projection step with a given pressure (no solve): forcing and correction only.  Used
 * to recompute the velocities of a step from a checkpointed pressure. */
int bcm_project_recompute(bcm_plan* plan, const bcm_project_in* in, const double* d_p,
                          bcm_project_out* out, void* stream);

/* Adjoint (reverse-mode derivative) of bcm_project: the transposed correction, the
 * transposed Poisson solve (A^T = V A V^{-1}, V = cell volumes), and the transposed face
 * interpolation, divergence and forcing.  Solver options as for the forward call. */
int bcm_project_adjoint(bcm_plan* plan, const bcm_adjoint_in* in, bcm_adjoint_out* out,
                        bcm_report* report, void* stream);

/* Momentum sub-step (Sec. 3, Eq. (substep1)) on single-level meshes with n >= 4 (other meshes:
 * BCM_ERR_UNSUPPORTED).  Explicit schemes are one pass; Crank-Nicolson iterates Jacobi sweeps
 * on its linear system from the Euler predictor, with a convergence check every check_every
 * iterations (solver options): report.n_inner = iterations, history = ||r|| / ||rhs|| at each
 * check, final_rel_res = the last of them, which is the residual of the iterate that the last
 * sweep started from (the returned iterate is one sweep further).  BCM_NOT_CONVERGED if cn_max_iter is reached first (output valid),
 * BCM_ERR_NONFINITE if a norm is not finite.  report may be NULL. */
int bcm_momentum(bcm_plan* plan, const bcm_momentum_in* in, bcm_momentum_out* out,
                 bcm_report* report, void* stream);

/* Forcing sub-step with Lagrangian particles (Sec. 3; Eqs. (ddeltai), (ddeltap)): every particle
 * interpolates u~ with the 3-point smoothed discrete delta function of Sec. 2.4 over the
 * 3 x 3 x 3 cells around the cell that holds it, U_p = sum_i u~_i prod_n phi((x_i,n - X_p,n)/h),
 * takes the constraint force F_p = (rho/dt)(U_s,p - U_p), and spreads it back with the same
 * weights: u* = u~ + (dt/rho) f, f_i = sum_p F_p prod_n phi(...) dV_p / h^3.  A particle's cell
 * is found on the finest level that has a cube there; its support must lie in cubes of that
 * level inside the domain.  The spread is added with atomics, so cells shared by several
 * particles are summed in no fixed order (results reproducible to rounding only).
 *   u_tilde / u_star  three device fields of the field type each (u_star written; must not
 *                     alias u_tilde)
 *   U_p, F_p          optional [n][3] device FP64 outputs (interpolated velocity, force), or NULL
 * Errors: BCM_ERR_INVALID_ARG (NULL or aliased fields, dt or rho not positive, 2^26 or more
 * particles (32 lanes each); or particles outside the mesh or with a support leaving their level or the domain: those are skipped, the
 * others' forcing is in u_star, and bcm_last_error gives the count), BCM_ERR_UNSUPPORTED (no
 * point-location tables: a level's cubes span more than 2^26 lattice positions).  The call
 * waits for the stream (it reads the skip count back). */
int bcm_ib_force(bcm_plan* plan, const bcm_particles* particles, const void* const u_tilde[3],
                 void* const u_star[3], double dt, double rho, double* U_p, double* F_p,
                 void* stream);

/* Lossy compression of an FP64 cell field for checkpoints (Sec. 6.4.1, Alg. "Compression
 * algorithm"): each cube transformed on its own by the CDF 5/3 wavelet (lifting along x, y, z,
 * log2(n) levels, symmetric extension at the cube faces), the coefficients quantised with one
 * uniform step (round half to even), the codes stored in groups of 32 at the group's bit width
 * (zigzag map), the cubes' streams concatenated behind a header of per-cube offsets:
 *   0 "BCMW" | 4 version 1 | 8 number of cubes | 12 n | 16 levels | 20 zero | 24 step (FP64) |
 *   32 (number of cubes + 1) u64 offsets relative to the data start | data: per cube the
 *   n^3/32 group widths (bytes, zero-padded to 4), then each group's w 32-bit words, code j at
 *   bits j w .. j w + w - 1 (little-endian).
 * Each cell of the decoded field differs from the original by at most gain * step / 2, gain =
 * the row-sum norm of the inverse transform (24.375 for n = 16).  Meshes with n >= 4 only
 * (else BCM_ERR_UNSUPPORTED).  The calls use the plan's Krylov vectors as scratch and wait for
 * the stream at their readbacks. */
/* Worst-case stream size of the plan's mesh (host only). */
int bcm_compress_bound(const bcm_plan* plan, size_t* bytes);
/* Compress the device field d_field (n_cubes * n^3 FP64) into d_stream (device, 8-byte aligned,
 * capacity bytes); *bytes = the stream's size.  BCM_ERR_INVALID_ARG if the buffer is too small
 * (the needed size is in *bytes; nothing past the header written), if step is not positive and
 * finite, or if a code would reach 2^30 (step too small for the field) or a value is not finite. */
int bcm_compress(bcm_plan* plan, const double* d_field, double step, void* d_stream,
                 size_t capacity, size_t* bytes, void* stream);
/* Decompress a stream of this mesh (device, 8-byte aligned, bytes long) into d_field.
 * BCM_ERR_INVALID_ARG if the header does not match the mesh or a cube's stream is malformed
 * (those cubes decode to zero). */
int bcm_decompress(bcm_plan* plan, const void* d_stream, size_t bytes, double* d_field,
                   void* stream);

/* Objective of the differentiable multi-step projection: the kinetic energy of a cell-centred
 * velocity field, J = (rho/2) sum_i V_i |u_i|^2 with V_i = h_i^3 the cell volume (the paper
 * states no normalisation for it; this is the discrete form on the mesh's cells), summed in
 * FP64 with a reduction whose order does not depend on the run (bitwise reproducible).
 *   u       three device fields of the plan's field type (cube-major, n_cubes * n^3 each)
 *   rho     density (> 0)
 *   J       host double, or NULL to skip the sum (then the call does not wait for the GPU)
 *   g_u     NULL, or three device fields of the field type that receive the cotangent
 *           g_scale * dJ/du_i = g_scale * rho * V_i * u_i (the seed of the reverse sweep)
 * Errors: BCM_ERR_INVALID_ARG (NULL field, rho <= 0, non-finite g_scale), BCM_ERR_WORKSPACE
 * (no workspace bound), BCM_ERR_NONFINITE (J not finite).  Uses the plan's workspace, so it
 * must not overlap other calls on the plan. */
int bcm_kinetic_energy(bcm_plan* plan, const void* const u[3], double rho, double g_scale,
                       double* J, void* const g_u[3], void* stream);

/* bcm_kinetic_energy for callers that cannot allocate device memory at the time of the call
 * (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same arguments, the same kernels and the same results bit for bit, but the reduction's
 * scratch (2048 partial sums and one scalar block, 16.5 KB) is a file-scope device array of the
 * library instead of the plan's workspace; the plan must still be bound (at set-up) for the
 * cube metadata.  The call allocates nothing: the first call on a device looks up that
 * device's copy of the array (held until the process ends); J is read back with a copy and a
 * stream synchronisation.  Every call on one GPU shares that GPU's array, so calls that
 * overlap on one GPU (other threads, other streams) race; nothing in the array needs clearing
 * (each call overwrites what it reads).  Errors as bcm_kinetic_energy, plus
 * BCM_ERR_UNSUPPORTED for a device index >= 64. */
int bcm_kinetic_energy_noalloc(bcm_plan* plan, const void* const u[3], double rho, double g_scale,
                               double* J, void* const g_u[3], void* stream);

/* Solve the pressure Poisson equation A p = b (Sec. 3) for a device FP64 right-hand side;
 * d_p holds the initial guess on entry if use_guess != 0 (else zero) and the solution on
 * exit. */
int bcm_poisson_solve(bcm_plan* plan, const double* d_b, double* d_p, int use_guess,
                      bcm_report* report, void* stream);

/* Apply the 7-point operator of the Poisson equation, in FP64: d_Ap = A d_p. */
int bcm_apply_laplacian(bcm_plan* plan, const double* d_p, double* d_Ap, void* stream);

/* Kernel timing: when enabled, every launch of the named kernel class is bracketed by HIP
 * events on the launch stream; bcm_timing_read returns the number of timed launches and
 * their summed duration (milliseconds), synchronising the events.  Classes are listed by
 * bcm_timing_name(i) for i = 0.. until it returns NULL.
 * The events themselves hold the stream for a few microseconds on each side of a timed
 * launch; bcm_timing_sample(plan, every) (every >= 1; 1 after bcm_timing_enable) times only
 * the first launch of each run of `every` launches of the class, to keep that cost out of a
 * timed region. */
int bcm_timing_enable(bcm_plan* plan, const char* kernel_class);
int bcm_timing_sample(bcm_plan* plan, int32_t every);
int bcm_timing_read(bcm_plan* plan, int64_t* launches, double* total_ms);
const char* bcm_timing_name(int i);

/* Bytes and cell counts the plan's mesh implies (for throughput reporting). */
int64_t bcm_mesh_cells(const bcm_mesh* mesh);

const char* bcm_status_string(int status);
const char* bcm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* BCM_H */
