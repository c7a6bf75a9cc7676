// Internal declarations of libmortarns: handle, device-side parameter blocks
// and kernel launchers.  Not part of the public C-ABI (include/mortarns.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "mortarns.h"

namespace mns {

constexpr int kMaxN = 6;  // points per direction: degree 2..5

// Per-quadrature-point linearization data (Sec. 2.3: the state enters the
// Jacobian only through these): a = u - u_ALE (d), grad u (d*d, row m = u_m),
// tau_u (1), tau_u * R (d).  16 values in 3D, 9 in 2D.
template <int DIM>
struct LinLayout {
  static constexpr int A = 0;
  static constexpr int GU = DIM;
  static constexpr int TAU = DIM + DIM * DIM;
  static constexpr int TR = TAU + 1;
  static constexpr int SIZE = TR + DIM;
};

// Per-quadrature-point metric of an iso-parametric cell (the Q_k
// interpolant of its node positions): K[p][m] = d xi_p / d x_m (p-major),
// JxW, and the mapping term of the Laplacian b_p = sum_m K[p][m] c_m with
// c_m = sum_pq (K K^T)_pq d^2 x_m / d xi_p d xi_q, so that
// lap u = sum_pq (K K^T)_pq d^2 u / d xi_p d xi_q - sum_p b_p d u / d xi_p.
// 13 values in 3D, 7 in 2D.
template <int DIM>
struct IsoLayout {
  static constexpr int K = 0;
  static constexpr int JXW = DIM * DIM;
  static constexpr int B = JXW + 1;
  static constexpr int SIZE = B + DIM;
};

// Per mortar point of an iso-parametric interface, stored per face side,
// segment slot and point at every rotor angle: the inverse Jacobians
// K[p][m] = d xi_p / d x_m of the own and the other side's interpolated map
// there, and cos, sin of the point's angle.
template <int DIM>
struct IsoMortarLayout {
  static constexpr int KO = 0;
  static constexpr int KX = DIM * DIM;
  static constexpr int C = 2 * DIM * DIM;
  static constexpr int S = C + 1;
  static constexpr int SIZE = S + 1;
};

// 1D tables: Lagrange basis on N Gauss-Lobatto nodes of [0,1] evaluated at the
// N Gauss points (the volume quadrature of every cell).
template <typename Real, int N>
struct Tab1D {
  Real V[N][N];   // V[q][a]  = L_a(x_q)
  Real D[N][N];   // D[q][a]  = L_a'(x_q)
  Real DD[N][N];  // DD[q][a] = L_a''(x_q)
  Real CD[N][N];  // CD[q][j]  = l_j'(x_q), l_j the Lagrange basis on the Gauss points
  Real CDD[N][N]; // CDD[q][j] = l_j''(x_q)
  Real x[N];      // Gauss points on [0,1]
  Real w[N];      // Gauss weights on [0,1]
};

// Structured annular geometry: cell and node numbering, radial spacing and
// physics constants of one launch.
template <typename Real>
struct Geom {
  long long ncells;     // both domains
  long long cell_off1;  // first stator cell
  long long node_off1;  // first stator node
  long long ndofs;
  int nth[2], nz;       // cells per ring of each domain, axial layers (1 in 2D)
  int ntd[2], nzn;      // theta node positions per ring of each domain, axial node planes (1 in 2D)
  int nr[2], nrn[2];    // radial cells / node rows per domain
  Real r0[2], dr[2];    // inner radius and radial cell size per domain
  Real dthd[2], dz;     // cell angle of each domain, layer height (1 in 2D)
  Real nu, omega;
  Real ct;              // BDF2 coefficient 3/(2 dt), 0 when steady
  Real ctau2;           // (1/dt)^2 in tau_u, 0 when steady
  Real h[2];            // element size per domain for each radial layer: see hcell
  const Real* hcell;    // [2][hstride] element size by (domain, radial layer)
  int hstride;
  const Real* trig;     // [nth[0] + nth[1]][N][2]: cos, sin of theta at (ring cell, Gauss point), rotor first
  // iso-parametric geometry (null on the polar path): per-point metric
  // [cell][point][IsoLayout::SIZE], physical point positions [cell][point][3]
  // and element sizes [cell] (the last two FP64, read by the state kernel)
  const Real* geo;
  const double* geox;
  const double* hiso;
};

// Mortar quadrature tables for the current rotor angle (Sec. 3.2).  Segment 0
// of stator face j spans [j dth, j dth + phi], segment 1 [j dth + phi, (j+1) dth];
// the rotor face on segment 0 is j - m - 1, on segment 1 it is j - m (mod n_theta).
template <typename Real, int N>
struct MortarTab {
  Real MV[2][2][N][N];  // [side][seg][q][a]: L_a at the side's theta-coordinate of mortar point q
  Real MD[2][2][N][N];  // d/dxi_theta of the same
  Real FV[2][N];        // [side][b]: L_b at the interface (xi_r = 1 rotor, 0 stator)
  Real FD[2][N];        // L_b' at the interface
  Real jxw[2][N][N];    // [seg][q_theta][q_z]: w R dtheta_seg (* w dz in 3D)
  Real tau_pen[2];      // penalty of the side's interface cells (Eq. EqPenalty)
  Real R;
  Real inv_rdth;        // 1 / (R dtheta)
  Real inv_dr[2];       // 1 / dr of the rotor and stator cells
  Real inv_dz;          // 1 / dz (3D), 0 in 2D
  int seg_active[2];
  int m;                // pairing offset, in [0, n_theta)
};

// Interface data of the general mortar kernels (unequal ring counts): every
// mortar segment is found and mapped inside the kernel from these values.
struct MortarGen {
  double theta_rot;                   // rotor angle
  const double* xnode;                // iso-parametric node positions [node][3] (material frame), or null
  const void* iso_geo;                // iso-parametric mortar point geometry (IsoMortarLayout, the launch's
                                      // precision) at the current angle, or null
  int npiece;                         // segment slots per face side in iso_geo
  double R;                           // interface radius
  double tau_pen[2];                  // penalty of the rotor and stator interface cells (Eq. EqPenalty)
  double inv_dr[2];                   // 1 / dr of the rotor and stator cells
  double inv_dz;                      // 1 / dz (3D), 0 in 2D
  double gll[kMaxN];                  // Gauss-Lobatto nodes on [0, 1]
  double ginv[kMaxN][kMaxN];          // 1 / (gll[j] - gll[q]) (0 for j = q)
  double FV[2][kMaxN], FD[2][kMaxN];  // L_b, L_b' at the interface (xi_r = 1 rotor, 0 stator)
};

struct Buffers {
  void* p = nullptr;
  size_t bytes = 0;
};

}  // namespace mns

struct mns_handle {
  mns_mesh_desc desc{};
  int dim = 0, k = 0, n = 0, nc = 0;
  int ntn = 0, nzn = 0, nz = 0;  // ntn: theta node positions of the rotor ring (= ntd[0])
  int nth[2] = {0, 0};           // cells per ring of each domain (equal unless n_theta_stator is set)
  int ntd[2] = {0, 0};           // theta node positions per ring of each domain
  double dthd[2] = {0, 0};       // cell angle of each domain
  bool equal_rings = true;       // nth[0] == nth[1]: two mortar segments per face at most
  int nrn[2] = {0, 0};
  int64_t ncells = 0, cell_off1 = 0, node_off1 = 0, nnodes = 0, ndofs = 0;
  double dth = 0, dz = 0;
  std::vector<double> gll, gx, gw;  // 1D rules
  std::vector<double> hcell;        // [2][hstride]
  int hstride = 0;
  double tau_pen[2] = {0, 0};
  bool rotated = false, linearized = false;
  double theta = 0, omega = 0;
  int m = 0;
  double phi = 0;
  // device buffers
  double* d_hcell64 = nullptr;
  float* d_hcell32 = nullptr;
  double* d_trig64 = nullptr;
  float* d_trig32 = nullptr;
  void* d_mtab64 = nullptr;  // MortarTab<double, N>
  void* d_mtab32 = nullptr;  // MortarTab<float, N>
  double* d_mtrig64 = nullptr;  // [n_theta][2][N][2] cos/sin at the mortar points of stator faces
  float* d_mtrig32 = nullptr;
  int64_t* d_cons = nullptr;    // constrained DoF indices (sorted)
  int64_t n_cons = 0;
  double* d_lin64 = nullptr;    // per-qp linearization data
  float* d_lin32 = nullptr;
  double* d_E64 = nullptr;      // local results [comp][local node][cell]
  float* d_E32 = nullptr;
  double* d_Em64 = nullptr;     // mortar cell-side local results [comp][local node][side*faces + face]
  float* d_Em32 = nullptr;
  double* d_hist = nullptr;     // BDF2 history / force of the current linearization (null when not given)
  double* d_force = nullptr;
  double* d_hist_buf = nullptr; // their buffers, allocated by the first linearization that passes them
  double* d_force_buf = nullptr;
  // solver workspace
  int ws_restart = 0;
  double* ws64 = nullptr;
  float* ws32 = nullptr;
  double* d_diag64 = nullptr;
  float* d_diag32 = nullptr;
  double* d_red = nullptr;      // reduction scratch
  double* d_gm = nullptr;       // FGMRES state on the device: partial sums, Hessenberg, rotations, scalars
  int gm_m = 0;                 // restart length d_gm was sized for
  double* d_step = nullptr;     // time-step work vectors (history, residual, rhs, increment, partials)
  double* d_state = nullptr;    // copy of the linearization state (multigrid injects it)
  // linearization source of the quad volume kernels, [0] FP64, [1] FP32:
  // 0 = B, the full per-point store d_lin64 / d_lin32 (a, grad u, tau, tau R);
  // 1 = C, tau and tau R per point (d_linc64 / d_linc32) with a and grad u
  // evaluated from the state (d_state / d_state32) inside the kernel
  int lin_src[2] = {0, 0};
  double* d_linc64 = nullptr;   // [cell][point][tau, tau R_x, tau R_y, tau R_z] (3D, degrees 2 and 3)
  float* d_linc32 = nullptr;
  float* d_state32 = nullptr;
  int lin_picard = 0;           // kind of the current linearization
  // iso-parametric geometry (mns_set_node_positions): node positions in the
  // material frame and the per-point tables rebuilt at every rotation
  bool iso = false;
  double tau_pen_polar[2] = {0, 0};  // penalty of the polar interface cells (restored by a reset)
  double* d_xnode = nullptr;    // [node][3]
  double* d_geo64 = nullptr;    // [cell][point][IsoLayout::SIZE]
  float* d_geo32 = nullptr;
  double* d_geox = nullptr;     // [cell][point][3] physical positions of the Gauss points
  double* d_hiso = nullptr;     // [cell] element size from the cell volume
  int* d_iso_flag = nullptr;    // set by the metric kernel where det J >= 0
  double* d_mgeo64 = nullptr;   // [face side][segment slot][mortar point][IsoMortarLayout::SIZE]
  float* d_mgeo32 = nullptr;
  int mgeo_pieces = 0;          // segment slots per face side
  long long lin_version = 0;    // incremented by every rotation and linearization
  void* mg = nullptr;           // multigrid hierarchy (mns_solver.hip)
  double* h_red = nullptr;      // pinned host mirror
  int red_cap = 0;
  bool diag_valid = false;
  // kernel configuration (mns_set_kernel_config): fused volume + mortar launch
  int fused = -1;
  // second stream and events of the concurrent launch (fused == 2), created at setup
  hipStream_t aux = nullptr;
  hipStream_t cap = nullptr;      // capture stream of the solver's graphs (default priority)
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // volume layout: 1 = lane quad per cell (3D, degrees 2 and 3), 0 = LDS planes
  int quad = 1;
  int picard = 0;               // linearization kind of the next mns_set_linearization (MNS_LIN_*)
  long long ws_gen = 0;         // incremented whenever the Krylov workspace is reallocated
  hipStream_t stream = nullptr;
  std::string err;
  // optional kernel timing (mns_enable_timing): event pairs per kernel class
  int timing_cap = 0;
  std::vector<hipEvent_t> ev[3];  // 2 * cap events per class: volume, mortar, other
  int ev_used[3] = {0, 0, 0};
};

namespace mns {

// One instance of a batched Jacobian application: its geometry and the
// device arrays of its handle; vectors of all instances are concatenated, the
// instance's slice starting at dof_off.
template <typename Real>
struct BatchItem {
  Geom<Real> G;
  const Real* lin;
  Real* E;
  Real* Em;
  const void* mtab;   // MortarTab<Real, N> of the handle
  const Real* mtrig;
  long long dof_off;
  int strip;          // local-result layout of the quad volume kernel
  const Real* iso_mg; // curved meshes: the mortar point table of the current angle
};

}  // namespace mns

// The instances of one dimension, degree and geometry kind (polar or
// curved) inside a batch: applied by one volume + mortar launch and one
// gather launch.
struct mns_batch_group {
  int dim = 0, k = 0;
  bool iso = false;
  std::vector<int> members;     // instance indices (handle order)
  // device: items (FP64, FP32), block prefix sums per precision: mortar,
  // volume (members + 1 each), gather (members + 1, shared)
  void* d_items64 = nullptr;
  void* d_items32 = nullptr;
  long long* d_prefix = nullptr;
  long long mtot[2] = {0, 0}, vtot[2] = {0, 0}, gtot = 0;
};

// Instances applied together (mns_batch_*), of any dimensions, degrees and
// geometry kinds: one group per (dimension, degree, kind), in the order of
// first appearance.
struct mns_batch {
  std::vector<mns_handle*> hs;
  long long ndofs = 0;
  std::vector<long long> offsets;
  std::vector<mns_batch_group> groups;
  // batched solver (mns_batch_solve): vector-block segmentation, workspace
  long long* d_seg = nullptr;   // block prefix per instance (count + 1), then dof offsets (count + 1)
  long long nvblk = 0;
  double* ws = nullptr;         // Krylov and Chebyshev vectors, diagonal
  float* ws32 = nullptr;
  int ws_m = 0;
  double* d_small = nullptr;    // solver state: partial sums, per-instance Arnoldi data and flags
  double* h_small = nullptr;    // pinned mirror of the per-instance flags
  size_t small_doubles = 0;     // capacity of d_small
  hipStream_t cap = nullptr;    // capture stream of the iteration graph
  // multigrid preconditioner: a batch over the instances' level-0 operators
  // when one of them is a Picard copy (else the batch itself is used)
  mns_batch* mg_fine = nullptr;
  std::vector<mns_handle*> mg_fine_hs;
  std::string err;
};

namespace mns {

int batch_build(mns_batch* b);
int batch_solve_impl(mns_batch* b, const double* rhs, double* x, const mns_solve_opts* o, mns_solve_report* reps,
                     hipStream_t s);
void batch_solver_free(mns_batch* b);
template <typename Real>
int launch_batch_jacobian(mns_batch* b, const Real* src, Real* dst, hipStream_t s);

// kernel launchers (mns_kernels.hip)
template <typename Real>
int launch_linearize(mns_handle* h, const double* state, const double* hist, const double* force,
                     Real* lin, hipStream_t s);
// d_linc64 / d_linc32 from d_lin64 (no-op where source C does not exist)
int launch_lin_compact(mns_handle* h, hipStream_t s);
template <typename Real>
int launch_jacobian(mns_handle* h, const Real* src, Real* dst, hipStream_t s);
// the same product with E and Em in the library's file-scope scratch array
template <typename Real>
int launch_jacobian_noalloc(mns_handle* h, const Real* src, Real* dst, hipStream_t s);
// device address (current device) and size of that array
int scratch_pointer(void** out, size_t* bytes);
int launch_residual(mns_handle* h, const double* state, double* res, hipStream_t s);
template <typename Real>
int launch_diagonal(mns_handle* h, Real* diag, hipStream_t s);
template <typename Real>
int launch_fill(Real* x, Real v, int64_t n, hipStream_t s);
template <typename Real>
int launch_constraints(const mns_handle* h, const Real* src, Real* dst, Real diag_value, int mode,
                       hipStream_t s);

// direct FP64 solve on the coarsest multigrid level (mns_coarse.hip):
// reconstruct the level's matrix by probing, factor and invert it
int coarse_setup(mns_handle* hc, void** state, hipStream_t s, int max_dofs);
void coarse_free(void* state);
double coarse_check_error(const void* state);
int assemble_matrix(mns_handle* h, double* A, long long lda, hipStream_t s);
template <typename Real>
int coarse_apply(const void* state, const Real* b, Real* x, hipStream_t s);
// the same solve for several instances in two launches: item j maps the
// entries [off, off + n) of b to those of x through its inverse, with
// coarse_parts(n) column-chunk partial sums of n values each in part; blk0
// and blk1 are its first blocks in the partial-sum launch and in the
// summation launch (items in block order; coarse_blocks gives the counts)
struct CoarseItem {
  const double* Ainv;
  long long lda;
  int n;
  long long off;
  double* part;
  long long blk0, blk1;
};
int coarse_parts(int n);
void coarse_blocks(int n, long long* part_blocks, long long* sum_blocks);
// Ainv, lda and n of a coarse solve (INVALID_ARG without one)
int coarse_item(const void* state, CoarseItem* it);
template <typename Real>
int coarse_apply_batch(const CoarseItem* items, int count, long long part_blocks, long long sum_blocks,
                       const Real* b, Real* x, hipStream_t s);

// vector casts (mns_solver.hip)
void mg_free(mns_handle* h);
int mg_levels(mns_handle* h, int* levels, hipStream_t s);
int mg_prolongate64(mns_handle* h, int level, const double* x, double* y, hipStream_t s);
int mg_restrict64(mns_handle* h, int level, const double* x, double* y, hipStream_t s);
int mns_bdf2_step_impl(mns_handle* h, double theta_next, double omega, const double* un, const double* unm1,
                       const double* force, double* u, const mns_step_opts* o, mns_step_report* rep, hipStream_t s);
int launch_cast_f64_f32(const double* a, float* b, int64_t n, hipStream_t s);
// h->d_diag64 / d_diag32 hold the diagonal of the current linearization
// (allocated and computed on first use, reused until it changes)
int cached_diagonal(mns_handle* h, hipStream_t s);
// multigrid of one instance of a batched solve: the hierarchy built and set
// up as mns_solve does (level-0 handle: the instance's or its Picard copy,
// with its lambda_max); x0 += the V-cycle's coarse-grid correction of the
// level-0 residual r0; Jacobian applications of its cycles
int mg_instance_setup(mns_handle* h, const mns_solve_opts* o, hipStream_t s, mns_handle** level0, double* lmax0);
template <typename Real>
int mg_instance_correction(mns_handle* h, const Real* r0, Real* x0, const mns_solve_opts* o, hipStream_t s);
void mg_instance_counts(mns_handle* h, int* v64, int* v32);
// the coarse-grid correction of every instance of a batch at once: each
// level's smoothing, residual, transfers, constraints and direct coarsest
// solves as batch launches (mns_solver.hip).  bmg_setup needs the hierarchies
// set up (mg_instance_setup) and a direct coarsest solve on each
// (UNSUPPORTED otherwise: the caller corrects per instance); level0[i] is
// instance i's level-0 handle.  bmg_correction: x0 += the correction of the
// level-0 residual r0 (its constrained rows zeroed in place), t0 work vector,
// all in the batch's layout.
struct BatchMG;
int bmg_setup(mns_batch* B, mns_handle* const* level0, const mns_solve_opts* o, bool f32, hipStream_t s,
              BatchMG** out);
template <typename Real>
int bmg_correction(BatchMG* M, Real* r0, Real* x0, Real* t0, hipStream_t s);
void bmg_counts(const BatchMG* M, int* v64, int* v32);
void bmg_free(BatchMG* M);
int launch_cast_f32_f64(const float* a, double* b, int64_t n, hipStream_t s);

// iso-parametric geometry (mns_iso.hip): node positions, fold check,
// element sizes and penalty; the per-point tables at the current angle
int iso_set_nodes(mns_handle* h, const double* xyz, int64_t n_nodes, hipStream_t s);
int iso_rotate(mns_handle* h, double theta, hipStream_t s);
// segment slots per face side of the mortar point table, and the table of
// the current angle (mns_kernels.hip)
int iso_mortar_pieces(const mns_handle* h);
int launch_iso_mortar_geo(mns_handle* h, hipStream_t s);

// host setup (mns_setup.cpp)
void rules_1d(int n, std::vector<double>& gll, std::vector<double>& gx, std::vector<double>& gw);
void lagrange_1d(const std::vector<double>& nodes, double t, double* L, double* dL, double* d2L);

int set_error(mns_handle* h, int code, const std::string& msg);

// timing hooks around a kernel launch (no-ops unless timing is enabled)
enum { TIMER_VOLUME = 0, TIMER_MORTAR = 1, TIMER_OTHER = 2 };
}  // namespace mns
