// Direct FP64 solve on the coarsest multigrid level (Sec. 3.4: a direct
// coarse-grid solver, with the level's matrix reconstructed column by column
// as in Alg. Alg-matrix, mortar columns included).
//
// Reconstruction: columns are recovered in groups from the matrix-free
// Jacobian itself.  Two columns whose row supports are disjoint can share one
// probe vector; the supports follow from the structure (all nodes of a cell
// couple, and all nodes of a rotor interface cell couple with all nodes of the
// stator interface cells that overlap it at the current angle), so a greedy
// distance-2 colouring of the nodes on the host gives the groups.  One probe
// per colour and component: J p, and every row of the result belongs to the
// one probed node that it couples to.  Constrained rows and columns come out
// as the identity, as in mns_apply_jacobian.
//
// Factorization: right-looking blocked LU with partial pivoting.  Blocks of
// 64 columns; each block is factored as sub-panels of 8 (4 above 4,096 rows)
// columns held in the registers of one 1024-thread workgroup, each followed
// by its row interchanges on the rest of the block, the triangular solve of
// its rows and the rank-8 update of the block's remaining columns; then the
// block's interchanges on every other column, the triangular solve of its 64
// rows and the FP64 tiled update of the trailing matrix.  The explicit inverse
// follows from P A = L U by blocked triangular solves with P as right-hand
// side.  Each coarse solve is then one FP64 matrix-vector product (two-stage,
// fixed order), which runs on many workgroups, unlike a triangular solve.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "mns_internal.hpp"

namespace mns {

constexpr int kNB = 64;        // panel width of the LU and of the blocked triangular solves
constexpr int kGemvRows = 256; // rows per workgroup of the matrix-vector product
// columns per workgroup (partial sums, summed in a second pass): 32 gives a
// 3456-row inverse 1,512 workgroups of 256 rows, enough loads in flight to
// read it at 3.7 TB/s (26 us; with 128 columns, 378 workgroups: 59 us)
constexpr int kGemvCols = 32;

// ---------------------------------------------------------------------------
// Probing
// ---------------------------------------------------------------------------

// p = 1 on component `comp` of the nodes of colour `color`, 0 elsewhere
__global__ void k_probe(const int* __restrict__ node_color, int color, int comp, int nc, long long nnodes,
                        double* __restrict__ p) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nnodes * nc) return;
  const long long node = i / nc;
  p[i] = (node_color[node] == color && (int)(i % nc) == comp) ? 1.0 : 0.0;
}

// A(row, col(row)) = y(row), col(row) = the probed node coupled to the row's
// node (owner table of the colour; -1: none) and the probed component
__global__ void k_probe_scatter(const int* __restrict__ owner, int comp, int nc, long long nnodes,
                                const double* __restrict__ y, double* __restrict__ A, long long lda) {
  const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nnodes * nc) return;
  const int a = owner[r / nc];
  if (a < 0) return;
  A[r + ((long long)a * nc + comp) * lda] = y[r];
}

__global__ void k_fill_mat(double* __restrict__ A, long long count, double v) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) A[i] = v;
}

__global__ void k_zero_mat(double* __restrict__ X, int n, long long ldx) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  const long long count = (long long)n * n;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride)
    X[i % n + (i / n) * ldx] = 0.0;
}

// ---------------------------------------------------------------------------
// Blocked LU with partial pivoting, column-major A (lda), in place
// ---------------------------------------------------------------------------

// Sub-panel [c0, c0 + w) (w <= PW) of rows [c0, n) factored by one
// workgroup of 1024 threads with the panel in registers: thread t owns rows
// c0 + t + 1024 r (r < R).  Per column: the pivot (largest magnitude,
// smallest row index among equals), the exchange of the two rows inside the
// sub-panel through LDS, the scaling of the column below the diagonal by the
// pivot's reciprocal and the rank-1 update of the sub-panel's later columns.
// piv[c] = pivot row of column c; *info = first zero pivot + 1.  Rows are
// exchanged only within the sub-panel; k_laswp applies the interchanges to
// the other columns.
constexpr int kLuThreads = 1024;

template <int R, int PW>
__global__ __launch_bounds__(kLuThreads) void k_lu_panel(double* __restrict__ A, int n, long long lda, int c0, int w,
                                                         int* __restrict__ piv, int* __restrict__ info) {
  __shared__ double wbest[kLuThreads / 64];
  __shared__ int wrow[kLuThreads / 64];
  __shared__ double prow[PW], srow[PW];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  double a[R][PW];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = c0 + t + kLuThreads * r;
#pragma unroll
    for (int j = 0; j < PW; ++j) a[r][j] = (i < n && j < w) ? A[i + (long long)(c0 + j) * lda] : 0.0;
  }
#pragma unroll
  for (int cc = 0; cc < PW; ++cc) {
    if (cc < w) {  // uniform across the workgroup
    const int c = c0 + cc;
    // pivot search over rows i >= c
    double best = -1.0;
    int bi = n;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = c0 + t + kLuThreads * r;
      if (i >= c && i < n) {
        const double v = fabs(a[r][cc]);
        if (v > best || (v == best && i < bi)) {
          best = v;
          bi = i;
        }
      }
    }
    for (int off = 32; off > 0; off >>= 1) {
      const double v = __shfl_xor(best, off, 64);
      const int ii = __shfl_xor(bi, off, 64);
      if (v > best || (v == best && ii < bi)) {
        best = v;
        bi = ii;
      }
    }
    if (lane == 0) {
      wbest[wv] = best;
      wrow[wv] = bi;
    }
    __syncthreads();
    double pv = wbest[0];
    int p = wrow[0];
#pragma unroll
    for (int q = 1; q < kLuThreads / 64; ++q)
      if (wbest[q] > pv || (wbest[q] == pv && wrow[q] < p)) {
        pv = wbest[q];
        p = wrow[q];
      }
    if (p >= n) p = c;  // no comparable candidate (NaN column): keep the row; info flags it below
    // exchange rows c and p inside the sub-panel
    const int tc = (c - c0) % kLuThreads, rc = (c - c0) / kLuThreads;
    const int tp = (p - c0) % kLuThreads, rp = (p - c0) / kLuThreads;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (t == tp && r == rp)
#pragma unroll
        for (int j = 0; j < PW; ++j) prow[j] = a[r][j];
      if (t == tc && r == rc)
#pragma unroll
        for (int j = 0; j < PW; ++j) srow[j] = a[r][j];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (t == tp && r == rp)
#pragma unroll
        for (int j = 0; j < PW; ++j) a[r][j] = srow[j];
      if (t == tc && r == rc)  // after the line above, so that p == c keeps the row
#pragma unroll
        for (int j = 0; j < PW; ++j) a[r][j] = prow[j];
    }
    if (t == 0) {
      piv[c] = p;
      if (!(pv > 0.0) && *info == 0) *info = c + 1;
    }
    // scale the column below the diagonal, update the later columns
    const double d = prow[cc];
    const double inv = d != 0.0 ? 1.0 / d : 0.0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = c0 + t + kLuThreads * r;
      if (i > c && i < n) {
        const double l = a[r][cc] * inv;
        a[r][cc] = l;
#pragma unroll
        for (int j = cc + 1; j < PW; ++j) a[r][j] -= l * prow[j];
      }
    }
    __syncthreads();  // prow, srow and the reduction slots are rewritten next column
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = c0 + t + kLuThreads * r;
#pragma unroll
    for (int j = 0; j < PW; ++j)
      if (i < n && j < w) A[i + (long long)(c0 + j) * lda] = a[r][j];
  }
}

// the interchanges of columns [c0, c0 + w) (piv) applied, in order, to the
// columns j in [j0, j1) outside [c0, c0 + w); one thread per column
__global__ void k_laswp(double* __restrict__ A, long long lda, int c0, int w, const int* __restrict__ piv, int j0,
                        int j1) {
  const int j = j0 + blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= j1 || (j >= c0 && j < c0 + w)) return;
  double* col = A + (long long)j * lda;
  for (int c = c0; c < c0 + w; ++c) {
    const int p = piv[c];
    if (p != c) {
      const double x = col[c];
      col[c] = col[p];
      col[p] = x;
    }
  }
}

// Triangular solve with the nb x nb (nb <= 64) diagonal block D of a factor
// held in F (rows/cols [k, k + nb)): X[k .. k + nb, j] = D^-1 X[k .. k + nb, j]
// for every column j in [j0, j1) of X (ldx).  lower: D unit lower triangular
// (forward); otherwise D upper triangular with its diagonal (backward).  One
// wavefront per column (lane = row of the block, the solved entry broadcast
// by a lane shuffle), D in LDS.
__global__ __launch_bounds__(256) void k_trsm_block(const double* __restrict__ F, long long ldf, int k, int nb,
                                                    double* __restrict__ X, long long ldx, int j0, int j1,
                                                    int lower) {
  __shared__ double D[kNB][kNB + 1];
  for (int e = threadIdx.x; e < nb * nb; e += blockDim.x) {
    const int r = e % nb, c = e / nb;
    D[r][c] = F[(k + r) + (long long)(k + c) * ldf];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int waves = blockDim.x >> 6;
  for (int j = j0 + blockIdx.x * waves + (threadIdx.x >> 6); j < j1; j += gridDim.x * waves) {
    double* col = X + (long long)j * ldx + k;
    double x = lane < nb ? col[lane] : 0.0;
    if (lower) {
      for (int c = 0; c + 1 < nb; ++c) {
        const double xc = __shfl(x, c, 64);
        if (lane > c && lane < nb) x -= D[lane][c] * xc;
      }
    } else {
      for (int c = nb - 1; c >= 0; --c) {
        const double xc = __shfl(x, c, 64) / D[c][c];
        if (lane == c) x = xc;
        else if (lane < c) x -= D[lane][c] * xc;
      }
    }
    if (lane < nb) col[lane] = x;
  }
}

// C[m x nn] -= L[m x kk] * U[kk x nn] (column-major, kk <= 64), 64 x 64 output
// tiles per workgroup of 256 threads, 4 x 4 outputs per thread
__global__ __launch_bounds__(256) void k_gemm_sub(const double* __restrict__ L, long long ldl,
                                                  const double* __restrict__ U, long long ldu, double* __restrict__ C,
                                                  long long ldc, int m, int nn, int kk) {
  __shared__ double Ls[kNB][kNB + 1];
  __shared__ double Us[kNB][kNB + 1];
  const int i0 = blockIdx.x * kNB, j0 = blockIdx.y * kNB;
  for (int e = threadIdx.x; e < kNB * kk; e += blockDim.x) {
    const int r = e % kNB, c = e / kNB;  // L tile: row r, column c < kk
    Ls[r][c] = i0 + r < m ? L[(i0 + r) + (long long)c * ldl] : 0.0;
    const int ur = e % kk, uc = e / kk;  // U tile: row ur < kk, column uc
    Us[ur][uc] = j0 + uc < nn ? U[ur + (long long)(j0 + uc) * ldu] : 0.0;
  }
  __syncthreads();
  const int tr = threadIdx.x % 16, tc = threadIdx.x / 16;
  double acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
  for (int q = 0; q < kk; ++q) {
    double l[4], u[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) l[a] = Ls[tr + 16 * a][q];
#pragma unroll
    for (int b = 0; b < 4; ++b) u[b] = Us[q][tc + 16 * b];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] += l[a] * u[b];
  }
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const int j = j0 + tc + 16 * b;
    if (j >= nn) continue;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int i = i0 + tr + 16 * a;
      if (i < m) C[i + (long long)j * ldc] -= acc[a][b];
    }
  }
}

// the row interchanges of the factorization, in order, as one permutation:
// row r of P A is row perm[r] of A (one workgroup; perm built in LDS)
constexpr int kMaxCoarseN = 8192;
__global__ __launch_bounds__(1024) void k_pivots_to_perm(const int* __restrict__ piv, int n, int* __restrict__ perm) {
  __shared__ int pm[kMaxCoarseN];
  for (int i = threadIdx.x; i < n; i += blockDim.x) pm[i] = i;
  __syncthreads();
  if (threadIdx.x == 0)
    for (int c = 0; c < n; ++c) {
      const int p = piv[c];
      const int x = pm[c];
      pm[c] = pm[p];
      pm[p] = x;
    }
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x) perm[i] = pm[i];
}

// X = P I: X(r, perm[r]) = 1, every other entry 0
__global__ void k_perm_identity(const int* __restrict__ perm, int n, double* __restrict__ X, long long ldx) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  const long long count = (long long)n * n;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) {
    const long long c = i / n, r = i % n;
    X[r + c * ldx] = perm[r] == c ? 1.0 : 0.0;
  }
}

// y = Ainv b in two stages: partial sums over column blocks of kGemvCols,
// then their sum in a fixed order (deterministic)
template <typename Real>
__global__ __launch_bounds__(kGemvRows) void k_gemv_part(const double* __restrict__ Ainv, long long lda, int n,
                                                         const Real* __restrict__ b, double* __restrict__ part) {
  const int i = blockIdx.x * kGemvRows + threadIdx.x;
  const int c0 = blockIdx.y * kGemvCols;
  __shared__ double bs[kGemvCols];
  for (int e = threadIdx.x; e < kGemvCols; e += blockDim.x) bs[e] = c0 + e < n ? (double)b[c0 + e] : 0.0;
  __syncthreads();
  if (i >= n) return;
  double s = 0.0;
  const int c1 = c0 + kGemvCols < n ? c0 + kGemvCols : n;
  for (int c = c0; c < c1; ++c) s += Ainv[i + (long long)c * lda] * bs[c - c0];
  part[(long long)blockIdx.y * n + i] = s;
}

// y[i] = sum over the parts of part[p][i] for the kSumRows rows of row block
// rb: the four wavefronts of the block sum a contiguous quarter of the parts
// each (loads of several parts in flight), then the quarters are added in
// order
constexpr int kSumRows = 64;
template <typename Real>
__device__ inline void gemv_sum_rows(const double* __restrict__ part, int n, int nparts, int rb, Real* __restrict__ y) {
  __shared__ double q[4][kSumRows];
  const int lane = threadIdx.x % kSumRows, w = threadIdx.x / kSumRows;
  const int i = rb * kSumRows + lane;
  const int per = (nparts + 3) / 4, p0 = w * per, p1 = p0 + per < nparts ? p0 + per : nparts;
  double s = 0.0;
  if (i < n) {
#pragma unroll 8
    for (int p = p0; p < p1; ++p) s += part[(long long)p * n + i];
  }
  q[w][lane] = s;
  __syncthreads();
  if (w == 0 && i < n) y[i] = (Real)(((q[0][lane] + q[1][lane]) + q[2][lane]) + q[3][lane]);
}

template <typename Real>
__global__ __launch_bounds__(4 * kSumRows) void k_gemv_sum(const double* __restrict__ part, int n, int nparts,
                                                           Real* __restrict__ y) {
  gemv_sum_rows<Real>(part, n, nparts, blockIdx.x, y);
}

// r = A x - y (check of the reconstruction), partial max |r| and max |y| per block
__global__ void k_check(const double* __restrict__ A, long long lda, int n, const double* __restrict__ x,
                        const double* __restrict__ y, double* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  __shared__ double se[256], sy[256];
  double e = 0.0, m = 0.0;
  if (i < n) {
    double s = 0.0;
    for (int c = 0; c < n; ++c) s += A[i + (long long)c * lda] * x[c];
    e = fabs(s - y[i]);
    m = fabs(y[i]);
  }
  se[threadIdx.x] = e;
  sy[threadIdx.x] = m;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      se[threadIdx.x] = fmax(se[threadIdx.x], se[threadIdx.x + off]);
      sy[threadIdx.x] = fmax(sy[threadIdx.x], sy[threadIdx.x + off]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[2 * blockIdx.x] = se[0];
    out[2 * blockIdx.x + 1] = sy[0];
  }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

// node index of (domain, theta, r, z) on handle h
static long long node_id(const mns_handle* h, int dom, int it, int ir, int iz) {
  return (dom ? h->node_off1 : 0) + it + (long long)h->ntd[dom] * (ir + (long long)h->nrn[dom] * iz);
}

// nodes of cell (dom, ct, cr, cz)
static void cell_nodes(const mns_handle* h, int dom, int ct, int cr, int cz, std::vector<long long>& out) {
  out.clear();
  const int k = h->k, nzl = h->dim == 3 ? k + 1 : 1;
  for (int c = 0; c < nzl; ++c)
    for (int b = 0; b <= k; ++b)
      for (int a = 0; a <= k; ++a) {
        int it = k * ct + a;
        if (it >= h->ntd[dom]) it -= h->ntd[dom];
        out.push_back(node_id(h, dom, it, k * cr + b, h->dim == 3 ? k * cz + c : 0));
      }
}

static int cfail(mns_handle* h, hipError_t e, const char* what) {
  return set_error(h, MNS_ERR_HIP, std::string("coarse solve ") + what + ": " + hipGetErrorString(e));
}

struct CoarseDirect {
  int n = 0;              // DoFs of the level
  long long lda = 0;
  double* A = nullptr;    // reconstructed matrix, then its LU factors (column-major)
  double* Ainv = nullptr; // explicit inverse
  double* part = nullptr; // partial sums of the matrix-vector product / check
  double* work = nullptr; // probe and result vectors
  int* piv = nullptr;
  int* perm = nullptr;    // the pivots as one row permutation
  int* info = nullptr;
  int* colors = nullptr;  // node colour
  int* owners = nullptr;  // [colour][node]: probed node coupled to the node, or -1
  int ncolors = 0;
  double check_err = 0;   // max |A x - J x| / max |J x| of the last reconstruction
};

void coarse_free(void* p) {
  auto* C = (CoarseDirect*)p;
  if (!C) return;
  for (void* q : {(void*)C->A, (void*)C->Ainv, (void*)C->part, (void*)C->work, (void*)C->piv, (void*)C->perm,
                  (void*)C->info, (void*)C->colors, (void*)C->owners})
    if (q) (void)hipFree(q);
  delete C;
}

// greedy distance-2 colouring of the nodes: two nodes share a colour only if
// no node couples to both (couplings: cell sharing, and mortar pairs of
// interface cells at the handle's current angle)
static void colour_nodes(const mns_handle* h, std::vector<int>& color, std::vector<int>& owners, int* ncolors) {
  const long long nn = h->nnodes;
  std::vector<std::vector<long long>> adj(nn);
  std::vector<long long> na, nb;
  const mns_mesh_desc& d = h->desc;
  const int nz = h->nz;
  auto couple = [&](const std::vector<long long>& x, const std::vector<long long>& y) {
    for (long long a : x) adj[a].insert(adj[a].end(), y.begin(), y.end());
  };
  for (int dom = 0; dom < 2; ++dom) {
    const int nr = dom ? d.n_r_stator : d.n_r_rotor;
    for (int cz = 0; cz < nz; ++cz)
      for (int cr = 0; cr < nr; ++cr)
        for (int ct = 0; ct < h->nth[dom]; ++ct) {
          cell_nodes(h, dom, ct, cr, cz, na);
          couple(na, na);
        }
  }
  // mortar pairs: a stator face and a rotor face whose angle ranges overlap
  // by more than the alignment tolerance (equal counts: stator face j meets
  // rotor faces j - m - 1, when the offset is not zero, and j - m)
  const double two_pi = 2.0 * M_PI, dts = h->dthd[1], dtr = h->dthd[0];
  const double tol = 1e-12 * std::min(dts, dtr);
  const double th = std::fmod(h->theta, two_pi) + (h->theta < 0 ? two_pi : 0.0);
  for (int cz = 0; cz < nz; ++cz)
    for (int j = 0; j < h->nth[1]; ++j) {
      cell_nodes(h, 1, j, 0, cz, na);
      for (int i = 0; i < h->nth[0]; ++i) {
        bool meet = false;
        if (h->equal_rings) {
          meet = i == (((j - h->m) % h->nth[0]) + h->nth[0]) % h->nth[0] ||
                 (h->phi > 0.0 && i == (((j - h->m - 1) % h->nth[0]) + h->nth[0]) % h->nth[0]);
        } else {
          for (int sh = -1; sh <= 1 && !meet; ++sh) {
            const double r0 = th + i * dtr + sh * two_pi;
            meet = std::min((j + 1) * dts, r0 + dtr) - std::max(j * dts, r0) > tol;
          }
        }
        if (!meet) continue;
        cell_nodes(h, 0, i, d.n_r_rotor - 1, cz, nb);
        couple(na, nb);
        couple(nb, na);
      }
    }
  for (auto& v : adj) {
    std::sort(v.begin(), v.end());
    v.erase(std::unique(v.begin(), v.end()), v.end());
  }
  color.assign(nn, -1);
  std::vector<std::vector<int>> claimed;  // [colour][node] = probed node coupled to it, or -1
  for (long long a = 0; a < nn; ++a) {
    int c = 0;
    for (;; ++c) {
      if (c == (int)claimed.size()) claimed.emplace_back(nn, -1);
      bool ok = true;
      for (long long b : adj[a])
        if (claimed[c][b] >= 0) {
          ok = false;
          break;
        }
      if (ok) break;
    }
    color[a] = c;
    for (long long b : adj[a]) claimed[c][b] = (int)a;
  }
  *ncolors = (int)claimed.size();
  owners.clear();
  for (auto& v : claimed) owners.insert(owners.end(), v.begin(), v.end());
}

// Dense reconstruction of the handle's Jacobian (rotated and linearized) into
// A (n x n, column-major, lda >= n): Alg. Alg-matrix by coloured probing.
// work: 2 n doubles; *colors / *owners: device tables (allocated here when
// null, reallocated when the colour count changes).  Enqueued on s; the
// tables are uploaded with a synchronization of s.
int assemble_dense(mns_handle* hc, double* A, long long lda, double* work, int** colors, int** owners, int* ncolors,
                   hipStream_t s) {
  const int n = (int)hc->ndofs;
  hipError_t e;
  std::vector<int> color, own;
  int ncol = 0;
  colour_nodes(hc, color, own, &ncol);
  if (!*colors && (e = hipMalloc((void**)colors, (size_t)hc->nnodes * sizeof(int))) != hipSuccess)
    return cfail(hc, e, "allocation");
  if (*owners && *ncolors != ncol) {
    (void)hipFree(*owners);
    *owners = nullptr;
  }
  if (!*owners && (e = hipMalloc((void**)owners, own.size() * sizeof(int))) != hipSuccess)
    return cfail(hc, e, "allocation");
  *ncolors = ncol;
  if ((e = hipMemcpyAsync(*colors, color.data(), color.size() * sizeof(int), hipMemcpyHostToDevice, s)) !=
          hipSuccess ||
      (e = hipMemcpyAsync(*owners, own.data(), own.size() * sizeof(int), hipMemcpyHostToDevice, s)) != hipSuccess ||
      (e = hipStreamSynchronize(s)) != hipSuccess)  // the host vectors go out of scope
    return cfail(hc, e, "tables");
  const long long nnodes = hc->nnodes;
  const int nc = hc->nc;
  const unsigned g = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(k_zero_mat, dim3(1024), dim3(256), 0, s, A, n, lda);
  double* p = work;
  double* y = work + n;
  int rc;
  for (int c = 0; c < ncol; ++c)
    for (int comp = 0; comp < nc; ++comp) {
      hipLaunchKernelGGL(k_probe, dim3(g), dim3(256), 0, s, (const int*)*colors, c, comp, nc, nnodes, p);
      if ((rc = launch_jacobian<double>(hc, p, y, s))) return rc;
      hipLaunchKernelGGL(k_probe_scatter, dim3(g), dim3(256), 0, s, (const int*)(*owners + (size_t)c * nnodes),
                         comp, nc, nnodes, (const double*)y, A, lda);
    }
  if ((e = hipGetLastError()) != hipSuccess) return cfail(hc, e, "probing");
  return MNS_OK;
}

template <int R, int PW>
static void launch_panel(CoarseDirect* C, int n, long long lda, int c0, int w, hipStream_t s) {
  hipLaunchKernelGGL((k_lu_panel<R, PW>), dim3(1), dim3(kLuThreads), 0, s, C->A, n, lda, c0, w, C->piv, C->info);
}

// one sub-panel factorization: rows [c0, n) need R = ceil((n - c0) / 1024)
// rows per thread; sub-panels are 8 columns wide up to 4,096 rows, 4 above
static void panel(CoarseDirect* C, int n, long long lda, int c0, int w, int pw, hipStream_t s) {
  const int R = (n - c0 + kLuThreads - 1) / kLuThreads;
  if (pw == 8) {
    switch (R) {
      case 1: launch_panel<1, 8>(C, n, lda, c0, w, s); break;
      case 2: launch_panel<2, 8>(C, n, lda, c0, w, s); break;
      case 3: launch_panel<3, 8>(C, n, lda, c0, w, s); break;
      default: launch_panel<4, 8>(C, n, lda, c0, w, s); break;
    }
  } else {
    switch (R) {
      case 1: launch_panel<1, 4>(C, n, lda, c0, w, s); break;
      case 2: launch_panel<2, 4>(C, n, lda, c0, w, s); break;
      case 3: launch_panel<3, 4>(C, n, lda, c0, w, s); break;
      case 4: launch_panel<4, 4>(C, n, lda, c0, w, s); break;
      case 5: launch_panel<5, 4>(C, n, lda, c0, w, s); break;
      case 6: launch_panel<6, 4>(C, n, lda, c0, w, s); break;
      case 7: launch_panel<7, 4>(C, n, lda, c0, w, s); break;
      default: launch_panel<8, 4>(C, n, lda, c0, w, s); break;
    }
  }
}

static unsigned trsm_grid(int cols) { return (unsigned)std::max(1, std::min(4096, (cols + 3) / 4)); }

// blocked LU of C->A in place, then C->Ainv = A^-1 from P A = L U
static int lu_invert(mns_handle* h, CoarseDirect* C, hipStream_t s) {
  const int n = C->n;
  const long long lda = C->lda;
  if (n > kMaxCoarseN) return set_error(h, MNS_ERR_UNSUPPORTED, "coarse level too large for the direct solve");
  const int pw = n <= 4 * kLuThreads ? 8 : 4;
  hipLaunchKernelGGL(k_fill_mat, dim3(1), dim3(64), 0, s, (double*)C->info, 1, 0.0);  // zero the info word
  for (int k = 0; k < n; k += kNB) {
    const int kend = std::min(n, k + kNB), nb = kend - k;
    // the block's columns, sub-panel by sub-panel
    for (int c0 = k; c0 < kend; c0 += pw) {
      const int w = std::min(pw, kend - c0), c1 = c0 + w;
      panel(C, n, lda, c0, w, pw, s);
      if (nb > w)
        hipLaunchKernelGGL(k_laswp, dim3((nb + 63) / 64), dim3(64), 0, s, C->A, lda, c0, w, (const int*)C->piv, k,
                           kend);
      if (c1 < kend) {
        hipLaunchKernelGGL(k_trsm_block, dim3(trsm_grid(kend - c1)), dim3(256), 0, s, (const double*)C->A, lda, c0,
                           w, C->A, lda, c1, kend, 1);
        if (n > c1)
          hipLaunchKernelGGL(k_gemm_sub, dim3((n - c1 + kNB - 1) / kNB, (kend - c1 + kNB - 1) / kNB), dim3(256), 0, s,
                             (const double*)(C->A + c1 + (long long)c0 * lda), lda,
                             (const double*)(C->A + c0 + (long long)c1 * lda), lda, C->A + c1 + (long long)c1 * lda,
                             lda, n - c1, kend - c1, w);
      }
    }
    // the block's interchanges on every other column, then the trailing update
    if (n > nb)
      hipLaunchKernelGGL(k_laswp, dim3((n + 255) / 256), dim3(256), 0, s, C->A, lda, k, nb, (const int*)C->piv, 0, n);
    const int rest = n - kend;
    if (rest > 0) {
      hipLaunchKernelGGL(k_trsm_block, dim3(trsm_grid(rest)), dim3(256), 0, s, (const double*)C->A, lda, k, nb, C->A,
                         lda, kend, n, 1);
      hipLaunchKernelGGL(k_gemm_sub, dim3((rest + kNB - 1) / kNB, (rest + kNB - 1) / kNB), dim3(256), 0, s,
                         (const double*)(C->A + kend + (long long)k * lda), lda,
                         (const double*)(C->A + k + (long long)kend * lda), lda, C->A + kend + (long long)kend * lda,
                         lda, rest, rest, nb);
    }
  }
  // X = P I, then L Y = X (forward, blocked), then U Ainv = Y (backward, blocked)
  double* X = C->Ainv;
  hipLaunchKernelGGL(k_pivots_to_perm, dim3(1), dim3(1024), 0, s, (const int*)C->piv, n, C->perm);
  hipLaunchKernelGGL(k_perm_identity, dim3(1024), dim3(256), 0, s, (const int*)C->perm, n, X, lda);
  const unsigned gcols = trsm_grid(n);
  for (int k = 0; k < n; k += kNB) {
    const int nb = std::min(kNB, n - k);
    hipLaunchKernelGGL(k_trsm_block, dim3(gcols), dim3(256), 0, s, (const double*)C->A, lda, k, nb, X, lda, 0, n, 1);
    const int rest = n - k - nb;
    if (rest > 0)
      hipLaunchKernelGGL(k_gemm_sub, dim3((rest + kNB - 1) / kNB, (n + kNB - 1) / kNB), dim3(256), 0, s,
                         (const double*)(C->A + (k + nb) + (long long)k * lda), lda, (const double*)(X + k), lda,
                         X + (k + nb), lda, rest, n, nb);
  }
  const int last = ((n - 1) / kNB) * kNB;
  for (int k = last; k >= 0; k -= kNB) {
    const int nb = std::min(kNB, n - k);
    hipLaunchKernelGGL(k_trsm_block, dim3(gcols), dim3(256), 0, s, (const double*)C->A, lda, k, nb, X, lda, 0, n, 0);
    if (k > 0)
      hipLaunchKernelGGL(k_gemm_sub, dim3((k + kNB - 1) / kNB, (n + kNB - 1) / kNB), dim3(256), 0, s,
                         (const double*)(C->A + (long long)k * lda), lda, (const double*)(X + k), lda, X, lda, k, n,
                         nb);
  }
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? MNS_OK : cfail(h, e, "factorization");
}

// Reconstruct the level's operator (handle hc, rotated and linearized) by
// probing, check it against one matrix-free product, and invert it.  The
// check reads two values back (synchronizes the stream).
int coarse_setup(mns_handle* hc, void** state, hipStream_t s, int max_dofs) {
  const long long n64 = hc->ndofs;
  if (n64 > max_dofs) return set_error(hc, MNS_ERR_UNSUPPORTED, "coarsest level too large for the direct solve");
  const int n = (int)n64;
  auto* C = (CoarseDirect*)*state;
  hipError_t e;
  if (!C || C->n != n) {
    coarse_free(C);
    *state = nullptr;
    C = new CoarseDirect();
    C->n = n;
    C->lda = n;
    const size_t nn = (size_t)n * n;
    const int parts = (n + kGemvCols - 1) / kGemvCols;
    if ((e = hipMalloc((void**)&C->A, nn * sizeof(double))) != hipSuccess ||
        (e = hipMalloc((void**)&C->Ainv, nn * sizeof(double))) != hipSuccess ||
        (e = hipMalloc((void**)&C->part, ((size_t)parts * n + 1024) * sizeof(double))) != hipSuccess ||
        (e = hipMalloc((void**)&C->work, 3 * (size_t)n * sizeof(double))) != hipSuccess ||
        (e = hipMalloc((void**)&C->piv, (size_t)n * sizeof(int))) != hipSuccess ||
        (e = hipMalloc((void**)&C->perm, (size_t)n * sizeof(int))) != hipSuccess ||
        (e = hipMalloc((void**)&C->info, 2 * sizeof(int))) != hipSuccess ||
        (e = hipMalloc((void**)&C->colors, (size_t)hc->nnodes * sizeof(int))) != hipSuccess) {
      coarse_free(C);
      return cfail(hc, e, "allocation");
    }
    *state = C;
  }
  int rc = assemble_dense(hc, C->A, C->lda, C->work, &C->colors, &C->owners, &C->ncolors, s);
  if (rc) return rc;
  double* y = C->work + n;
  const unsigned g = (unsigned)((n + 255) / 256);
  // check: A x = J x for one vector with every entry nonzero
  {
    std::vector<double> xh(n);
    for (int i = 0; i < n; ++i) xh[i] = (double)(i % 97 + 1) / 97.0 - 0.5;
    double* xv = C->work + 2 * (size_t)n;
    if ((e = hipMemcpyAsync(xv, xh.data(), n * sizeof(double), hipMemcpyHostToDevice, s)) != hipSuccess)
      return cfail(hc, e, "check");
    if ((rc = launch_jacobian<double>(hc, xv, y, s))) return rc;
    hipLaunchKernelGGL(k_check, dim3(g), dim3(256), 0, s, (const double*)C->A, C->lda, n, (const double*)xv,
                       (const double*)y, C->part);
    std::vector<double> out(2 * g);
    if ((e = hipMemcpyAsync(out.data(), C->part, out.size() * sizeof(double), hipMemcpyDeviceToHost, s)) !=
            hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
      return cfail(hc, e, "check");
    double em = 0, ym = 0;
    for (unsigned b = 0; b < g; ++b) {
      em = std::max(em, out[2 * b]);
      ym = std::max(ym, out[2 * b + 1]);
    }
    C->check_err = ym > 0 ? em / ym : em;
    if (!(C->check_err < 1e-10))
      return set_error(hc, MNS_ERR_HIP, "coarse matrix reconstruction does not reproduce the operator (" +
                                            std::to_string(C->check_err) + ")");
  }
  if ((rc = lu_invert(hc, C, s))) return rc;
  int info = 0;
  if ((e = hipMemcpyAsync(&info, C->info, sizeof(int), hipMemcpyDeviceToHost, s)) != hipSuccess ||
      (e = hipStreamSynchronize(s)) != hipSuccess)
    return cfail(hc, e, "factorization");
  if (info) return set_error(hc, MNS_ERR_HIP, "coarse matrix is singular (zero pivot " + std::to_string(info) + ")");
  return MNS_OK;
}

double coarse_check_error(const void* state) { return state ? ((const CoarseDirect*)state)->check_err : -1.0; }

// dense reconstruction for the C-ABI (mns_assemble_matrix): temporary tables
// and work vectors, synchronizes the stream
int assemble_matrix(mns_handle* h, double* A, long long lda, hipStream_t s) {
  double* work = nullptr;
  int *colors = nullptr, *owners = nullptr, ncol = 0;
  hipError_t e = hipMalloc((void**)&work, 2 * (size_t)h->ndofs * sizeof(double));
  if (e != hipSuccess) return cfail(h, e, "allocation");
  int rc = assemble_dense(h, A, lda, work, &colors, &owners, &ncol, s);
  e = hipStreamSynchronize(s);
  if (!rc && e != hipSuccess) rc = cfail(h, e, "assembly");
  (void)hipFree(work);
  if (colors) (void)hipFree(colors);
  if (owners) (void)hipFree(owners);
  return rc;
}

// x = A^-1 b in FP64 (b, x in the cycle's precision)
template <typename Real>
int coarse_apply(const void* state, const Real* b, Real* x, hipStream_t s) {
  const auto* C = (const CoarseDirect*)state;
  const int n = C->n;
  const int parts = (n + kGemvCols - 1) / kGemvCols;
  hipLaunchKernelGGL(k_gemv_part<Real>, dim3((n + kGemvRows - 1) / kGemvRows, parts), dim3(kGemvRows), 0, s,
                     (const double*)C->Ainv, C->lda, n, b, C->part);
  hipLaunchKernelGGL(k_gemv_sum<Real>, dim3((n + kSumRows - 1) / kSumRows), dim3(4 * kSumRows), 0, s,
                     (const double*)C->part, n, parts, x);
  return hipGetLastError() == hipSuccess ? MNS_OK : MNS_ERR_HIP;
}
template int coarse_apply<double>(const void*, const double*, double*, hipStream_t);
template int coarse_apply<float>(const void*, const float*, float*, hipStream_t);

int coarse_item(const void* state, CoarseItem* it) {
  const auto* C = (const CoarseDirect*)state;
  if (!C || !C->Ainv) return MNS_ERR_INVALID_ARG;
  it->Ainv = C->Ainv;
  it->lda = C->lda;
  it->n = C->n;
  return MNS_OK;
}

// x = Ainv b for several instances, in the two stages of coarse_apply
// (partial sums over column chunks of kGemvCols, then the chunks summed in
// order): one launch of (item, row block, chunk) blocks and one of
// (item, row block) blocks
int coarse_parts(int n) { return (n + kGemvCols - 1) / kGemvCols; }

void coarse_blocks(int n, long long* part_blocks, long long* sum_blocks) {
  const long long rows = (n + kGemvRows - 1) / kGemvRows;
  *part_blocks = rows * coarse_parts(n);
  *sum_blocks = (n + kSumRows - 1) / kSumRows;
}

__device__ inline int coarse_find(const CoarseItem* items, int count, long long b, bool second) {
  int a = 0, z = count - 1;  // last item whose first block is at or before b
  while (a < z) {
    const int mid = (a + z + 1) >> 1;
    if ((second ? items[mid].blk1 : items[mid].blk0) <= b) a = mid;
    else z = mid - 1;
  }
  return a;
}

template <typename Real>
__global__ __launch_bounds__(kGemvRows) void k_gemv_batch_part(const CoarseItem* __restrict__ items, int count,
                                                               const Real* __restrict__ b) {
  const CoarseItem& it = items[coarse_find(items, count, blockIdx.x, false)];
  const long long local = (long long)blockIdx.x - it.blk0;
  const int rows = (it.n + kGemvRows - 1) / kGemvRows;
  const int rb = (int)(local % rows), p = (int)(local / rows);
  const int i = rb * kGemvRows + threadIdx.x;
  const int c0 = p * kGemvCols;
  const Real* bi = b + it.off;
  __shared__ double bs[kGemvCols];
  for (int e = threadIdx.x; e < kGemvCols; e += blockDim.x) bs[e] = c0 + e < it.n ? (double)bi[c0 + e] : 0.0;
  __syncthreads();
  if (i >= it.n) return;
  double s = 0.0;
  const int c1 = c0 + kGemvCols < it.n ? c0 + kGemvCols : it.n;
  for (int c = c0; c < c1; ++c) s += it.Ainv[i + (long long)c * it.lda] * bs[c - c0];
  it.part[(long long)p * it.n + i] = s;
}

template <typename Real>
__global__ __launch_bounds__(4 * kSumRows) void k_gemv_batch_sum(const CoarseItem* __restrict__ items, int count,
                                                                 Real* __restrict__ x) {
  const CoarseItem& it = items[coarse_find(items, count, blockIdx.x, true)];
  gemv_sum_rows<Real>(it.part, it.n, (it.n + kGemvCols - 1) / kGemvCols, (int)((long long)blockIdx.x - it.blk1),
                      x + it.off);
}

template <typename Real>
int coarse_apply_batch(const CoarseItem* items, int count, long long part_blocks, long long sum_blocks,
                       const Real* b, Real* x, hipStream_t s) {
  if (count == 0) return MNS_OK;
  hipLaunchKernelGGL(k_gemv_batch_part<Real>, dim3((unsigned)part_blocks), dim3(kGemvRows), 0, s, items, count, b);
  hipLaunchKernelGGL(k_gemv_batch_sum<Real>, dim3((unsigned)sum_blocks), dim3(4 * kSumRows), 0, s, items, count, x);
  return hipGetLastError() == hipSuccess ? MNS_OK : MNS_ERR_HIP;
}
template int coarse_apply_batch<double>(const CoarseItem*, int, long long, long long, const double*, double*,
                                        hipStream_t);
template int coarse_apply_batch<float>(const CoarseItem*, int, long long, long long, const float*, float*,
                                       hipStream_t);

}  // namespace mns
