/*
 * mortarns.h -- C-ABI of libmortarns.so: matrix-free Jacobian of the
 * linearized SUPG/PSPG-stabilized ALE incompressible Navier-Stokes operator on
 * a rotor/stator pair of annular Q_k-Q_k meshes coupled by mortar face
 * integrals, on one AMD Instinct MI355X (gfx950).
 *
 * Operator (arXiv 2608.27423):
 *   - weak form with mortar interface terms: Sec. 2.1, Eqs. EqMortarPre,
 *     EqMortarDiff (SIPG), EqPenalty (Hillewaert penalty), EqMortarMass
 *     (strong-DG mass term), Eq-NSweakWmortar;
 *   - SUPG/PSPG stabilization with the Tezduyar parameter: Sec. 2.2, Eqs.
 *     Eq-NSweakComplete, Eq-strong-residual, Eq-stab-param;
 *   - Newton system and the stabilized Jacobian blocks: Sec. 2.3, Eqs.
 *     Eq-Newton-method, Eq-Newton-matrix, Eq-discrete-1..4;
 *   - rigid rotor rotation and mortar segments with a mapped reference
 *     quadrature: Sec. 3.1, Sec. 3.2, Eq. Eq-Jacobian;
 *   - diagonal by unit-vector columns of the mortar terms: Alg. Alg-diagonal.
 *
 * Conventions fixed by this library where the paper leaves them open: jump and
 * normal are taken per side (jump = own - other, n = own outward normal, rotor
 * +e_r, stator -e_r); tau_u is frozen in the Jacobian; h = 2 sqrt(A/pi) (2D),
 * (6V/pi)^(1/3) (3D); Gauss-Lobatto nodes with k+1 Gauss points per direction;
 * exact polar geometry, or iso-parametric cells from node positions
 * (mns_set_node_positions); no-slip on every external wall and one pinned pressure
 * DoF (stator node at theta index 0, outermost radius, z index 0).
 *
 * Vector layout (every vector argument): DoF index = node*(d+1) + comp, comps
 * (u_x, u_y[, u_z], p) in the lab frame's Cartesian axes.  Per domain, nodes are
 * lexicographic with theta fastest (periodic, k*n_theta positions), then r
 * (k*n_r+1 positions), then z (k*n_z+1, 3D only).  The rotor block comes first.
 * Rotor nodes are numbered in the rotor's material frame, so rotation never
 * permutes a vector.
 *
 * Memory and streams: every vector pointer is DEVICE memory on the current HIP
 * device, contiguous, 8-byte aligned (double) or 4-byte aligned (float).  The
 * caller owns all vectors; the library owns the handle and its workspace.
 * mns_setup_mesh allocates the geometry and angle tables, the per-point
 * linearization store, the local-result buffers and a second stream with its
 * events; mns_set_linearization allocates only on the first call that passes
 * a history or force vector; the first mns_solve allocates the Krylov
 * workspace.  mns_rotate_rotor, mns_set_linearization (after that first call)
 * and mns_apply_* allocate nothing.  Work is enqueued on the stream argument
 * (a hipStream_t, NULL = default stream) in stream order; the calls that take
 * a stream neither synchronize the host nor the device, except mns_solve,
 * mns_bdf2_step, mns_batch_solve and mns_autotune_kernel_config, which
 * synchronize their stream.  A handle's tables are rewritten in the order of
 * the stream passed to mns_rotate_rotor / mns_set_linearization: work on
 * another stream that reads the handle must be ordered against those calls by
 * the caller (events), as for any buffer shared between streams.
 *
 * Errors: every int-returning call returns MNS_OK (0) or a negative MNS_ERR_*
 * code; the handle keeps a message readable with mns_last_error.  No C++
 * exception crosses this interface.  A handle must not be used from two host
 * threads at once.
 */
#ifndef MORTARNS_H
#define MORTARNS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  MNS_OK = 0,
  MNS_ERR_INVALID_ARG = -1,   /* bad size, ordering, null or misaligned pointer */
  MNS_ERR_HIP = -2,           /* a HIP runtime call failed */
  MNS_ERR_NOT_LINEARIZED = -3,/* mns_set_linearization has not been called */
  MNS_ERR_NOT_CONVERGED = -4, /* mns_solve stopped at maxit; x holds the last iterate */
  MNS_ERR_UNSUPPORTED = -5,   /* valid request the library does not implement */
  MNS_ERR_NO_ROTATION = -6    /* mns_rotate_rotor has not been called */
};

enum { MNS_F64 = 0, MNS_F32 = 1 };
/* preconditioner choice of mns_solve_opts.precond besides -1 / MNS_F64 / MNS_F32 */
enum { MNS_PRECOND_MG = 2, MNS_PRECOND_MG64 = 3 };
/* linearization kind (mns_set_linearization_kind, mns_solve_opts.mg_coarse_linearization) */
enum { MNS_LIN_NEWTON = 0, MNS_LIN_PICARD = 1 };

typedef struct mns_handle mns_handle;

/* Mesh and physics description (Sec. 2, Sec. 3.1).  Rotor annulus
 * r_in < r < r_interface, stator annulus r_interface < r < r_out, with n_theta
 * azimuthal cells in the rotor ring and n_theta_stator (default: n_theta) in
 * the stator ring, n_r_rotor resp. n_r_stator radial cells, and in 3D n_z
 * axial layers on [0, height] (equal on both sides). */
typedef struct {
  int dim;               /* 2 or 3 */
  int degree;            /* k >= 2: 2..5 in 2D, 2..4 in 3D */
  double r_in, r_interface, r_out;
  double height;         /* 3D only */
  int n_theta, n_r_rotor, n_r_stator, n_z; /* n_z ignored in 2D */
  double nu;             /* kinematic viscosity > 0 */
  double penalty_F;      /* F of Eq. EqPenalty, > 0 (1 .. 10 typical) */
  int penalty_side_rule; /* 0: each side its own cell tau_k; 1: max of both sides */
  int steady;            /* 1: no time derivative; 0: BDF2 with constant dt */
  double dt;             /* time step (transient only) */
  int n_theta_stator;    /* cells per ring of the stator; 0 (or n_theta): the equal interface counts of
                            Sec. 2.1 / Sec. 3.1.  Another count lifts that restriction (the extension named
                            in Sec. 3.1 and Sec. 5): a face may then meet several faces of the other side,
                            every intersection being one mortar segment (at most 4:1 either way).  Such meshes
                            support the Jacobian, residual, diagonal and mns_solve with the Jacobi-Chebyshev
                            preconditioner; multigrid, batching and the fused launch need equal counts */
} mns_mesh_desc;

/* Create a handle: validates the description, builds the 1D tables, the
 * constraint list and the per-layer element sizes, and allocates device
 * tables.  The rotor angle is unset until mns_rotate_rotor.
 * Errors: INVALID_ARG (k < 2, n_theta < 3, radii not increasing, nu <= 0,
 * ...), UNSUPPORTED (degree outside the compiled set), HIP. */
int mns_setup_mesh(const mns_mesh_desc* desc, void* stream, mns_handle** out);

/* Total DoFs and rotor DoFs (the rotor block is [0, n_rotor)). */
int mns_n_dofs(const mns_handle* h, int64_t* n_total, int64_t* n_rotor);

/* Rigid rotation x = R(theta) x0 of the rotor (Sec. 3.1) and mesh velocity
 * u_ALE = omega e_z x x in rotor cells.  Rebuilds the mortar segments of every
 * stator face (one when aligned to 1e-12 of a cell angle, else two), the
 * mapped quadrature tables of Sec. 3.2 and the rotated geometry tables, all in
 * FP64 (cast copies for FP32), with one kernel enqueued on `stream` (three
 * on curved meshes, which also rebuild the per-point metric and the mortar
 * points' inverse Jacobians): work enqueued earlier on `stream` still sees the
 * old tables, later work the new ones.  Allocates nothing and does not synchronize, so it can be captured
 * into a graph (the angle is a kernel argument).  Invalidates the
 * linearization (the next apply needs mns_set_linearization).
 * Errors: INVALID_ARG (non-finite theta or omega), HIP. */
int mns_rotate_rotor(mns_handle* h, double theta, double omega, void* stream);

/* Fix the state (u, p) at which the Jacobian is taken (Eq. Eq-Newton-method)
 * and precompute per quadrature point the convective velocity a = u - u_ALE,
 * grad u, tau_u (Eq. Eq-stab-param) and tau_u R (Eq. Eq-strong-residual), in
 * FP64 and FP32.  u_hist: BDF2 history term (-4 u^n + u^(n-1)) / (2 dt) in the
 * vector layout (pressure slots ignored), or NULL; ignored when steady.
 * force: body force f in the vector layout, or NULL.  The arrays are read on
 * `stream` by the enqueued work; the library keeps copies (a history buffer
 * and a force buffer are allocated by the first call that passes them and
 * kept; every other call allocates nothing).
 * Errors: NO_ROTATION, INVALID_ARG (null or misaligned state), HIP. */
int mns_set_linearization(mns_handle* h, const double* state, const double* u_hist, const double* force,
                          void* stream);

/* Iso-parametric geometry (the mesh mapping of Sec. 2.1: each cell is the
 * Q_k interpolant of its Gauss-Lobatto node positions).  xyz: HOST array of
 * n_nodes x 3 doubles (x, y, z; z ignored in 2D), one row per node in the
 * node order of the vector layout, rotor nodes in the rotor's material frame
 * (the rotation x = R(theta) x0 of Sec. 3.1 is applied by mns_rotate_rotor);
 * the library copies it.  Interface nodes (rotor outermost and stator
 * innermost node rows) must sit at their polar positions on the circle
 * r = r_interface, where the mortar integrals stay (exact circle, exact
 * normal, JxW = w R dtheta_seg dz of Eq. Eq-Jacobian); the gradients there go
 * through each cell's interpolated map.  Volume integrals, element sizes
 * (from the interpolated cell volumes) and the interface penalty (Eq.
 * EqPenalty, from the interpolated measures of the ring-0, layer-0
 * interface cell of each side) follow the interpolated cells.  xyz NULL
 * returns to the exact polar geometry.  The Jacobian, residual, diagonal,
 * matrix reconstruction, allocation-free apply, mns_solve and mns_bdf2_step
 * (every preconditioner) support this geometry; it always
 * runs the LDS-plane volume layout with the mortar kernel in its own launch
 * (mns_kernel_config's volume layout, fused launch and linearization source
 * do not apply); the multigrid V-cycle builds curved coarse levels from
 * these positions (mns_mg_levels); batching needs the polar geometry
 * (UNSUPPORTED).  Allocates the node and per-point metric tables on first
 * use (13 values per Gauss point in 3D, 7 in 2D, FP64 and FP32) and
 * synchronizes the stream.  Clears the rotation and the linearization (call
 * mns_rotate_rotor and mns_set_linearization again) and frees a multigrid
 * hierarchy built for the previous geometry.
 * Errors: INVALID_ARG (n_nodes not the mesh's node count, non-finite values,
 * an interface node off its polar position, a cell whose map folds: det J
 * zero or of the wrong orientation at a Gauss-Lobatto point), HIP. */
int mns_set_node_positions(mns_handle* h, const double* xyz, int64_t n_nodes, void* stream);

/* Kind of the linearization that the next mns_set_linearization builds.
 * MNS_LIN_NEWTON (default): the Newton Jacobian of Sec. 2.3.  MNS_LIN_PICARD:
 * the Picard (Oseen) operator of the same residual, i.e. the Newton blocks
 * without the derivative of the convection velocity (the reaction term
 * (du . grad) u) and without the derivative of the SUPG weight (tau R . (du .
 * grad) v); a = u - u_ALE, tau_u and the mortar terms are unchanged.  With no
 * history and no force, J_picard(u) u equals the residual R(u).  The multigrid
 * preconditioner may linearize its coarse levels this way
 * (mns_solve_opts.mg_coarse_linearization).
 * Errors: INVALID_ARG (unknown kind). */
int mns_set_linearization_kind(mns_handle* h, int kind);

/* dst = J src: the stabilized Jacobian of Sec. 2.3 with the mortar face terms
 * of Sec. 2.1 at the current angle and linearization.  Constrained columns
 * read as zero; constrained rows give dst = src.  precision MNS_F64: src and
 * dst are double*; MNS_F32: float* and the whole product runs in FP32.  src
 * and dst must not overlap.  Allocates nothing.
 * Errors: NOT_LINEARIZED, INVALID_ARG, HIP. */
int mns_apply_jacobian(mns_handle* h, int precision, const void* src, void* dst, void* stream);

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): the product of
 * mns_apply_jacobian (same arguments, same result bit for bit) whose volume
 * and mortar kernels keep their local results in one library-owned device
 * array of MNS_NOALLOC_SCRATCH_BYTES instead of the handle's buffers.  The
 * array is part of the library's code object: every GPU that the library
 * runs on holds its own copy until the process ends, and this call allocates
 * nothing.  Meshes whose local results exceed the array are refused
 * (UNSUPPORTED): the local results take 4 (k+1)^3 values per 3D cell plus
 * the same per interface face side, so in FP64 the 32,768-cell degree-2
 * workload (64 x 8 x 32 cells per domain, 31.9 MB) fits.  Every call
 * on one GPU shares that GPU's array, which keeps the last call's contents:
 * calls that overlap in time on one GPU (different streams or threads) race
 * and must be serialized by the caller.
 * Errors: NOT_LINEARIZED, INVALID_ARG, UNSUPPORTED (mesh too large), HIP. */
#define MNS_NOALLOC_SCRATCH_BYTES (32u << 20)
int mns_apply_jacobian_noalloc(mns_handle* h, int precision, const void* src, void* dst, void* stream);

/* A = J as a dense matrix (column-major, n = n_total rows and columns,
 * leading dimension lda >= n, device memory of the caller): every column of
 * the current Jacobian, mortar columns included, reconstructed from the
 * matrix-free product (Alg. Alg-matrix): nodes are coloured so that no row
 * couples to two nodes of one colour, and one product per colour and
 * component yields all their columns.  Constrained rows and columns are
 * those of the identity.  This is the reconstruction behind the direct
 * coarse-grid solve of the multigrid preconditioner; meant for small meshes
 * (n <= 32,768) and tests.  Allocates temporary tables and synchronizes the
 * stream.  Errors: NOT_LINEARIZED, INVALID_ARG, UNSUPPORTED (n too large), HIP. */
int mns_assemble_matrix(mns_handle* h, double* A, int64_t lda, void* stream);

/* res = R(state): the discrete nonlinear residual of Eq. Eq-NSweakWmortar plus
 * the SUPG/PSPG terms of Eq. Eq-NSweakComplete (tau_u from `state`), with the
 * history and force given at the last mns_set_linearization; constrained rows
 * are zero.  Allocates nothing.  Errors: NO_ROTATION, INVALID_ARG, HIP. */
int mns_apply_residual(mns_handle* h, const double* state, double* res, void* stream);

/* diag = diagonal of J (volume columns plus Alg. Alg-diagonal for the mortar
 * terms); constrained rows are 1.  Errors: NOT_LINEARIZED, INVALID_ARG, HIP. */
int mns_compute_diagonal(mns_handle* h, int precision, void* diag, void* stream);

typedef struct {
  double rtol;        /* stop at ||rhs - J x||_2 <= rtol ||rhs||_2 (default 1e-8) */
  int restart;        /* FGMRES restart length m (default 50) */
  int maxit;          /* max outer iterations in total (default 2000) */
  int precond;        /* -1: none; MNS_F64 or MNS_F32: one Jacobi-Chebyshev polynomial whose vmults run in
                         that precision; MNS_PRECOND_MG: geometric multigrid V-cycle (below) with FP32
                         smoothing; MNS_PRECOND_MG64: the same V-cycle entirely in FP64 */
  int cheb_degree;    /* Chebyshev polynomial degree; smoothing degree per step in the V-cycle (default 4) */
  double cheb_range;  /* ratio lambda_max / lambda_min of the Chebyshev interval (default 30) */
  int eig_iters;      /* power iterations for lambda_max of D^-1 J (default 20) */
  int mg_levels;      /* V-cycle: most levels including the mesh itself, 0 = as many as the mesh allows */
  int mg_smooth_degree;     /* V-cycle: Chebyshev smoothing degree before and after the correction (default 2) */
  double mg_smooth_range;   /* V-cycle: smoothing interval [lambda_max / range, lambda_max] (default 5) */
  int mg_coarse_degree;     /* V-cycle: Chebyshev degree on the coarsest level (default 16) */
  int mg_coarse_linearization; /* V-cycle: MNS_LIN_NEWTON (default) or MNS_LIN_PICARD for levels 1, 2, ... */
  int mg_fine_linearization;   /* V-cycle on the mesh's own level: MNS_LIN_NEWTON (default) smooths with the
                                  handle's operator; MNS_LIN_PICARD with a Picard copy of it at the same state
                                  (one more set of per-point data).  FGMRES always applies the handle's operator */
  int use_graph;               /* 1 (default): one whole FGMRES iteration (preconditioner, FP64 Jacobian,
                                  Gram-Schmidt passes, Hessenberg and Givens update, next basis vector; every
                                  launch reads the column index from the device state) is captured once per call
                                  into a HIP graph on a library stream and replayed on `stream`; the host reads
                                  the state back once per chunk of iterations.  0: the same launches one by one.
                                  Ignored by mns_solve while kernel timing is enabled.  Same arithmetic either way */
  double cheb_lambda_factor;   /* every Chebyshev interval (the polynomial preconditioner here and in mns_batch_solve,
                                  the V-cycle smoothers and coarse polynomial): upper end = this factor times the
                                  power-iteration estimate of lambda_max, lower end = upper / (cheb_range or
                                  mg_smooth_range).  The estimate converges from below; a factor a little above 1
                                  keeps the top of the spectrum inside the interval (default 1.05; valid range
                                  [1, 4]) */
  int mg_coarse_direct;        /* V-cycle, coarsest level (always FP64): 1 (default): direct solve with the level's
                                  matrix reconstructed column by column from its Jacobian (Alg. Alg-matrix, mortar
                                  columns included) and inverted by LU with partial pivoting on the device, when the
                                  level has at most 8,192 DoFs (a Chebyshev polynomial otherwise); 0: Chebyshev of
                                  degree mg_coarse_degree */
} mns_solve_opts;

typedef struct {
  int iterations;         /* outer FGMRES iterations taken */
  int restarts;
  int status;             /* MNS_OK or MNS_ERR_NOT_CONVERGED */
  double rel_residual;    /* true ||rhs - J x||_2 / ||rhs||_2, recomputed in FP64 */
  double lambda_max;      /* power-iteration estimate (before cheb_lambda_factor) */
  double seconds;         /* wall time of the call */
  int vmults_f64, vmults_f32;
} mns_solve_report;

/* Fill opts with the defaults above. */
void mns_default_solve_opts(mns_solve_opts* opts);

/* Multigrid preconditioner (precond = MNS_PRECOND_MG or MNS_PRECOND_MG64),
 * degree 2 or 3.  Levels: the mesh itself; for degree 3 then the degree-2
 * space on the same mesh (polynomial level); then degree-2 meshes with
 * n_theta, n_r_rotor, n_r_stator (and n_z in 3D) halved while all stay even
 * (nested polar meshes: every coarse cell is 2 x 2 (x 2) fine cells of the
 * same map).  On a curved mesh (mns_set_node_positions) every coarse level
 * is curved too: a halved mesh takes every other node position of the level
 * above, the degree-2 level of a degree-3 mesh the Q3 interpolant of each
 * cell at its Q2 nodes, and interface nodes stay at their polar positions on
 * the circle; a coarse cell whose map folds fails the solve with
 * INVALID_ARG.  On every level:
 * the operator of mns_apply_jacobian with mortar faces at the same rotor
 * angle, linearized at the finest state evaluated at the level's nodes (Newton
 * or, with mg_coarse_linearization = MNS_LIN_PICARD, Picard on the coarse
 * levels); FP32 Jacobi-Chebyshev smoothing of degree
 * mg_smooth_degree on [lambda_max / mg_smooth_range, lambda_max] of D^-1 J
 * before and after the coarse correction; Chebyshev of degree
 * mg_coarse_degree on the coarsest level.  Transfers: prolongation = the
 * coarse field evaluated at the fine nodes, restriction = its transpose;
 * constrained entries are zero after each transfer.  The hierarchy is built on
 * the first V-cycle solve and relinearized when the state or the angle
 * changed. */
int mns_mg_levels(mns_handle* h, int* levels);

/* y = P_level x: prolongation from multigrid level `level`+1 to `level`
 * (level 0 = the mesh of h); x has the coarse level's n_total doubles, y the
 * fine level's.  For inspection and tests; builds the hierarchy if needed.
 * Errors: INVALID_ARG (no such level), UNSUPPORTED (degree not 2 or 3), HIP. */
int mns_mg_prolongate(mns_handle* h, int level, const double* x, double* y, void* stream);

/* y = P_level^T x: the restriction the V-cycle applies, from level `level` to
 * `level`+1 (x has the fine level's n_total doubles, y the coarse level's),
 * computed direction by direction (theta, r, z).  For inspection and tests;
 * builds the hierarchy if needed.  Errors: as mns_mg_prolongate. */
int mns_mg_restrict(mns_handle* h, int level, const double* x, double* y, void* stream);

/* Solve J x = rhs with flexible GMRES in FP64 (classical Gram-Schmidt with one
 * reorthogonalization), right-preconditioned by a Jacobi-Chebyshev polynomial
 * of D^-1 J whose vmults run in the precision opts->precond, or by the
 * multigrid V-cycle.  x holds the
 * initial guess on entry and the iterate on return; rhs is any device vector
 * and, since constrained rows of J are identity rows, the constrained entries
 * of the solution equal those of rhs.  Synchronizes the stream.  The first
 * call (and any call with a larger restart) allocates the Krylov workspace
 * (2 * restart + 9 FP64 vectors plus 5 FP32 vectors); with use_graph each call
 * instantiates and frees one graph of the preconditioner.
 * Errors: NOT_LINEARIZED, INVALID_ARG, NOT_CONVERGED (report filled), HIP. */
int mns_solve(mns_handle* h, const double* rhs, double* x, const mns_solve_opts* opts, mns_solve_report* report,
              void* stream);

/* One implicit time step of the transient ALE problem (Sec. 2.2 with the
 * rotor rotation of Sec. 3.1): BDF2 with constant step dt (from the mesh
 * description, which must be transient) and Newton's method on the nodal
 * residual, every linear step solved by mns_solve.
 *   1. the rotor is rotated to theta_next (mns_rotate_rotor semantics);
 *   2. history term h = (-4 u_n + u_nm1) / (2 dt), so that c_t u + h is the
 *      BDF2 derivative with c_t = 3 / (2 dt).  With u_nm1 == NULL the first
 *      step uses h = -(3 / (2 dt)) u_n: backward Euler with step 2 dt / 3.
 *      Rotor nodes keep their material numbering, so the history needs no
 *      remapping after the rotation;
 *   3. u = u_next (initial guess; it must hold the Dirichlet values); repeat:
 *      linearize at u, R = residual(u) (constrained rows 0), stop when
 *      ||R||_2 <= max(newton_atol, newton_rtol ||R(u_0)||_2), else solve
 *      J d = -R (constrained entries of d are 0) and set u += a d with the
 *      first a in 1, 1/2, ..., 1/256 for which ||R(u + a d)||_2 <=
 *      (1 - 1e-4 a) ||R(u)||_2 (the smallest when none is).
 * u_n, u_nm1, force and u_next are device vectors of n_total doubles; u_next
 * is overwritten with the last iterate.  The Jacobian freezes tau at the
 * current iterate (the operator of mns_apply_jacobian).  The first call
 * allocates five work vectors.  Synchronizes the stream.
 * Errors: INVALID_ARG (steady mesh, bad pointers or options), HIP,
 * NOT_CONVERGED (max_newton reached or a linear solve failed; u_next holds
 * the last iterate and the report is filled). */
typedef struct {
  double newton_rtol;     /* default 1e-8 */
  double newton_atol;     /* default 1e-13 */
  int max_newton;         /* default 8 */
  mns_solve_opts linear;  /* default mns_default_solve_opts with rtol 1e-6 */
} mns_step_opts;

typedef struct {
  int newton_iterations;  /* linear solves taken */
  int linear_iterations;  /* FGMRES iterations summed over the solves */
  int status;             /* MNS_OK or MNS_ERR_NOT_CONVERGED */
  double residual0;       /* ||R||_2 at the initial guess */
  double residual;        /* ||R||_2 at the returned iterate */
  double seconds;         /* wall time of the call */
  int line_search_halvings; /* step halvings summed over the Newton iterations */
} mns_step_report;

void mns_default_step_opts(mns_step_opts* opts);
int mns_bdf2_step(mns_handle* h, double theta_next, double omega, const double* u_n, const double* u_nm1,
                  const double* force, double* u_next, const mns_step_opts* opts, mns_step_report* report,
                  void* stream);

/* Batched Jacobian application (many rotor/stator instances at once).  A
 * batch holds `count` handles of any dimensions and degrees (any mesh sizes,
 * angles, viscosities, steady or transient, polar or curved geometry; equal
 * interface counts), each rotated and linearized before mns_batch_create.
 * Vectors of a batch are the instances' vectors concatenated in handle order
 * (mns_batch_n_dofs gives the total length).  The instances of one
 * dimension, degree and geometry kind (polar, curved) form a launch group:
 * mns_batch_apply_jacobian computes
 * dst_i = J_i src_i for every instance with, per group, one launch for all
 * its volume cells and mortar faces (in the block order of the
 * single-instance fused launch, the instance of a block found from block
 * prefix sums) and one gather launch;
 * the arithmetic is that of mns_apply_jacobian, so every slice equals the
 * instance's own product.  Later rotations and linearizations of the handles
 * are seen by later batch calls; a handle must outlive its batches.  The
 * batch allocates its tables at creation and nothing per call.
 * Errors: INVALID_ARG (null, misaligned vectors), NOT_LINEARIZED,
 * UNSUPPORTED (unequal interface counts), HIP; creation errors are reported on
 * handles[0], apply errors by mns_batch_last_error. */
typedef struct mns_batch mns_batch;
int mns_batch_create(mns_handle* const* handles, int count, mns_batch** batch);
int mns_batch_n_dofs(const mns_batch* batch, int64_t* n_total);
int mns_batch_apply_jacobian(mns_batch* batch, int precision, const void* src, void* dst, void* stream);
const char* mns_batch_last_error(const mns_batch* batch);

/* Batched FGMRES: solve J_i x_i = rhs_i for every instance of the batch at
 * once (concatenated vectors, as mns_batch_apply_jacobian).  The instances run
 * in lockstep: every iteration is one batched preconditioner application, one
 * batched FP64 Jacobian application and batched Gram-Schmidt reductions
 * (blocks of one instance each, per-instance sums in a fixed order); the
 * Hessenberg and Givens updates, the power iteration and the Chebyshev scalars
 * run per instance on the device, so that with use_graph one iteration is a
 * graph replay and the host synchronizes once per chunk of iterations and
 * once per restart cycle.  Preconditioner:
 * opts->precond -1, MNS_F64 or MNS_F32 (Jacobi-Chebyshev of degree
 * cheb_degree <= 32 on [lambda_i / cheb_range, lambda_i], lambda_i by power
 * iteration per instance); restart <= 200 (up to 31 the Gram-Schmidt
 * kernels hold all coefficients in registers and read each basis vector once
 * per pass; longer restarts process the columns in chunks of 32);
 * MNS_PRECOND_MG or MNS_PRECOND_MG64: the V-cycle of mns_solve on every
 * instance, every level batched: on each level the smoothing polynomials
 * (degree mg_smooth_degree <= 32, per-instance diagonals and lambda_max) and
 * the residual run as batch launches over the instances' operators of that
 * level, the restriction, prolongation and constrained rows as one launch
 * per step, and the FP64 direct coarsest solves of the instances whose
 * hierarchy ends there as one launch (hierarchies of different depths mix).
 * Without a direct coarsest solve on every instance (mg_coarse_direct 0, or
 * a coarsest level too large for it) the finest level stays batched and each
 * instance's coarse-grid correction runs through its own cycle.  Every
 * instance's hierarchy needs two or more levels (degree 3, or a mesh that
 * can be halved: UNSUPPORTED otherwise); each handle keeps its hierarchy as
 * after mns_solve.  An
 * instance that has converged
 * keeps its iterate while the others continue.  reports (count entries, or
 * NULL) receive per-instance iterations, relative residuals and lambda_max
 * (0 without a preconditioner; the finest level's with multigrid).
 * The first call allocates (2 * restart + 12) FP64 and 8 FP32 batch vectors
 * and the solver state (a few KB per instance); a call with a larger restart
 * or degree grows them.  Each instance's diagonal is its handle's, computed
 * (and on the first use allocated) once per linearization and shared with
 * mns_solve, so repeated solves of one linearization give identical iterates.
 * Multigrid builds or updates each instance's hierarchy as mns_solve does
 * and allocates, for the call, the batched levels' vectors and tables (and,
 * when the finest levels are Picard copies, a batch over those copies).
 * Synchronizes the stream.
 * Errors: INVALID_ARG, UNSUPPORTED (multigrid on a one-level hierarchy),
 * NOT_CONVERGED (some instance reached maxit), HIP. */
int mns_batch_solve(mns_batch* batch, const double* rhs, double* x, const mns_solve_opts* opts,
                    mns_solve_report* reports, void* stream);
void mns_batch_destroy(mns_batch* batch);

/* Kernel configuration of the Jacobian application (tuning knobs; every
 * setting computes the same product).  fused_launch = 1: volume cells and
 * mortar faces are integrated in one launch (3D degree 2: volume blocks
 * first; otherwise mortar blocks first); 0: two launches on the caller's
 * stream; 2: two launches, the
 * mortar kernel on a second stream of the library (default priority) joined
 * back to the caller's stream before the gather; -1 (default): 1 below
 * 262,144 cells, 2 from there on.  In FP64 at degree 2 with the quad
 * layout the volume blocks of every mode keep their Gauss-point values in
 * LDS (two wavefronts per SIMD); in the fused launch the mortar blocks then
 * take fewer faces so that both kinds fit the same LDS.  volume_layout = 1
 * (default): in 3D with degree 2 or 3 a quad of four lanes owns a cell and
 * the theta contractions exchange values between lanes without LDS; 0:
 * (k+1)^2 lanes per cell (nine for degree 2, sixteen for degree 3) with the
 * r and theta contractions staged through LDS, the layout used in 2D and for
 * degree >= 4 whatever the setting.  lin_source_f64 / lin_source_f32: where
 * the volume kernel takes the linearization data of a point (Sec. 2.3: the
 * advection velocity a = u - w, grad u, tau and the strong residual R), per
 * precision.  0 (default): source B, all 16 values per Gauss point from the
 * store written by mns_set_linearization; 1: source C, only tau and tau R per
 * point (4 values) from that store, a and grad u evaluated from the state
 * inside the kernel like the increment (more arithmetic, a quarter of the
 * per-point bytes).  Source C exists with the quad layout for 3D degree 2
 * (both precisions) and degree 3 (FP32); elsewhere source B is used whatever
 * the setting.  The two sources give the same operator up to rounding.
 * Takes effect on the next apply call.
 * Errors: INVALID_ARG. */
typedef struct {
  int fused_launch;
  int volume_layout;
  int lin_source_f64;
  int lin_source_f32;
} mns_kernel_config;
int mns_set_kernel_config(mns_handle* h, const mns_kernel_config* cfg);
int mns_get_kernel_config(const mns_handle* h, mns_kernel_config* cfg);

/* Autotuner of the launch configuration: times `reps` FP64 applications of
 * every launch mode (fused_launch 0, 1, 2), in 3D with degree 2 or 3 both
 * volume layouts, and with the quad layout both linearization sources where
 * source C exists, on the handle's own mesh and linearization, and sets the
 * fastest; then, with that launch mode and layout, times `reps` FP32
 * applications with each FP32 linearization source and sets the faster
 * (written to *chosen when non-null).  All configurations compute the same
 * product up to rounding; the choice depends on the mesh size (tail of the
 * fused launch against the cost of a second stream) and on the balance of
 * memory traffic and arithmetic.  Allocates four work vectors for the
 * duration of the call and synchronizes the stream.
 * Errors: INVALID_ARG (reps outside 1..1000, kernel timing enabled),
 * NOT_LINEARIZED, HIP. */
int mns_autotune_kernel_config(mns_handle* h, int reps, mns_kernel_config* chosen, void* stream);

/* Kernel timing for measurement.  mns_enable_timing(h, capacity) makes every
 * later mns_apply_jacobian record a pair of HIP events around each of its
 * kernels on the launch stream (capacity = max recorded launches per kernel
 * class; the events are created here, not in the apply call); capacity 0
 * turns timing off.  mns_read_timing synchronizes on those events, returns
 * the summed milliseconds and launch counts of the volume, mortar and other
 * (fill, constraint) kernels since the last read, and resets them.
 * Errors: INVALID_ARG, HIP. */
typedef struct {
  double ms_volume, ms_mortar, ms_other;
  int n_volume, n_mortar, n_other;
} mns_timing;
int mns_enable_timing(mns_handle* h, int capacity);
int mns_read_timing(mns_handle* h, mns_timing* out);

/* Measurement: rate of a read-dominated stream on the current device, the
 * practical HBM ceiling for the roofline figures.  Reads read_bytes from src
 * (seen as `ratio` contiguous blocks of 32-byte words) and writes
 * read_bytes / ratio to dst (word o = sum of word o of every block), `reps`
 * times after one untimed pass, timed with HIP events on `stream`, for each
 * of eight launch shapes (1,024 to 8,192 workgroups of 256 threads, one or
 * two words per thread and step); *gbs = the best (bytes read + bytes
 * written) per second / 1e9.  src and dst are device
 * buffers of at least read_bytes and read_bytes / ratio bytes, 32-byte
 * aligned.  Synchronizes the stream.
 * Errors: INVALID_ARG (sizes, alignment, ratio outside 1..64), HIP. */
int mns_stream_bandwidth(const void* src, void* dst, int64_t read_bytes, int ratio, int reps, void* stream,
                         double* gbs);

/* Last error message of the handle ("" if none).  Never NULL. */
const char* mns_last_error(const mns_handle* h);

/* Release the handle and all its device memory (synchronizes its stream). */
void mns_destroy(mns_handle* h);

#ifdef __cplusplus
}
#endif
#endif
