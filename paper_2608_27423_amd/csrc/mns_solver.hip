// Flexible GMRES(m) in FP64 with a Jacobi-Chebyshev polynomial preconditioner
// whose Jacobian applications run in FP32 (mixed) or FP64 (plain).  The outer
// Krylov basis, the Hessenberg reduction and the true residual are FP64.
//
// Orthogonalization: classical Gram-Schmidt with one reorthogonalization pass
// when the projected norm drops below 0.7 of the original (DGKS criterion);
// each pass is one fused multi-dot kernel and one fused multi-axpy/norm kernel
// with a deterministic two-stage reduction.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "mns_batch_vec.hpp"
#include "mns_internal.hpp"

int mns_build_handle(const mns_mesh_desc* d, hipStream_t stream, mns_handle* h);

namespace mns {

constexpr int kRedBlocks = 1024;  // partial-sum blocks of the reductions
constexpr int kRedThreads = 256;

template <typename From, typename To>
__global__ void k_cast(const From* __restrict__ a, To* __restrict__ b, long long n) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) b[i] = (To)a[i];
}

// block-level sum of K values per thread into out[blockIdx.x * K + i]; the
// loops run over the full register array with a predicate, so that the
// array stays in registers (a loop bounded by K indexes it dynamically)
template <int MAXK>
__device__ inline void block_sum_store(double (&v)[MAXK], int K, double* out) {
  __shared__ double s[kRedThreads / 64][MAXK];
  const int lane = threadIdx.x % 64, wid = threadIdx.x / 64;
#pragma unroll
  for (int i = 0; i < MAXK; ++i) {
    if (i < K) {
      double x = v[i];
      for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
      if (lane == 0) s[wid][i] = x;
    }
  }
  __syncthreads();
  if (threadIdx.x < K) {
    double t = 0;
    for (int w = 0; w < kRedThreads / 64; ++w) t += s[w][threadIdx.x];
    out[blockIdx.x * K + threadIdx.x] = t;
  }
}

constexpr int kDotK = 32;  // register width of the fused Gram-Schmidt kernels

// partial dots of w with V_0 .. V_{K-1} (contiguous, stride n); with self,
// entry K is w . w (K + self <= 32 per launch)
__global__ __launch_bounds__(kRedThreads) void k_multidot(const double* __restrict__ V, long long n, int K,
                                                          const double* __restrict__ w, double* __restrict__ part,
                                                          int self) {
  double acc[kDotK];
#pragma unroll
  for (int i = 0; i < kDotK; ++i) acc[i] = 0;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += stride) {
    const double wr = w[r];
#pragma unroll
    for (int i = 0; i < kDotK; ++i) {
      if (i < K) acc[i] += V[(long long)i * n + r] * wr;
      if (self && i == K) acc[i] += wr * wr;
    }
  }
  block_sum_store<kDotK>(acc, K + self, part);
}

// second stage: out[i] = sum over blocks of part[b * K + i], fixed order
__global__ void k_reduce_parts(const double* __restrict__ part, int nblocks, int K, double* __restrict__ out) {
  __shared__ double s[256];
  for (int i = blockIdx.x; i < K; i += gridDim.x) {
    double t = 0;
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x) t += part[(long long)b * K + i];
    s[threadIdx.x] = t;
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
      if (threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[i] = s[0];
    __syncthreads();
  }
}

__global__ void k_scale_copy(const double* __restrict__ a, double s, double* __restrict__ b, long long n) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) b[i] = s * a[i];
}

// r = b - Ax (in place on Ax), partial ||r||^2
__global__ __launch_bounds__(kRedThreads) void k_residual(const double* __restrict__ b, double* __restrict__ Ax,
                                                          long long n, double* __restrict__ part) {
  double acc[1] = {0};
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const double r = b[i] - Ax[i];
    Ax[i] = r;
    acc[0] += r * r;
  }
  block_sum_store<1>(acc, 1, part);
}

// x += sum_i y_i Z_i
__global__ void k_update_x(const double* __restrict__ Z, long long n, int K, const double* __restrict__ y,
                           double* __restrict__ x) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += stride) {
    double s = x[r];
    for (int i = 0; i < K; ++i) s += y[i] * Z[(long long)i * n + r];
    x[r] = s;
  }
}

// Chebyshev start: r = b ; d = D^-1 b / theta ; x = d
template <typename Real>
__global__ void k_cheb_init(const Real* __restrict__ b, const Real* __restrict__ diag, Real inv_theta,
                            Real* __restrict__ r, Real* __restrict__ d, Real* __restrict__ x, long long n,
                            const Real* __restrict__ sub) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    // sub: the polynomial applied to b - sub (a residual formed on the fly)
    const Real bi = sub ? b[i] + Real(-1) * sub[i] : b[i];
    const Real di = inv_theta * bi / diag[i];
    r[i] = bi;
    d[i] = di;
    x[i] = di;
  }
}

// Chebyshev step: r -= Jd ; d = c1 d + c2 D^-1 r ; x += d
template <typename Real>
__global__ void k_cheb_step(Real* __restrict__ r, const Real* __restrict__ Jd, const Real* __restrict__ diag,
                            Real c1, Real c2, Real* __restrict__ d, Real* __restrict__ x, long long n) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const Real ri = r[i] - Jd[i];
    const Real di = c1 * d[i] + c2 * ri / diag[i];
    r[i] = ri;
    d[i] = di;
    x[i] += di;
  }
}

// y = D^-1 J v / scale (power iteration), partial ||y||^2
__global__ __launch_bounds__(kRedThreads) void k_power_step(const double* __restrict__ Jv,
                                                            const double* __restrict__ diag, double* __restrict__ y,
                                                            long long n, double* __restrict__ part) {
  double acc[1] = {0};
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const double v = Jv[i] / diag[i];
    y[i] = v;
    acc[0] += v * v;
  }
  block_sum_store<1>(acc, 1, part);
}

// ---------------------------------------------------------------------------
// FGMRES iteration on the device.  The Gram-Schmidt coefficients, the
// Hessenberg column, the Givens rotations, the residual estimate and the
// convergence flag live in device memory, and every kernel of an iteration
// reads the column index j from there, so one iteration is the same sequence
// of launches for every j: it is captured once per solve into a graph and
// replayed, and the host reads the state back once per chunk of iterations.
// Layout of the state (doubles, restart m, P = m + 2): partial sums
// [kRedBlocks][P], hcol[P], h2[P], cs[m], sn[m], g[m + 1], H[(m + 1) m]
// (row-major, H[i m + j]), y[m], misc[16].
// ---------------------------------------------------------------------------
enum {
  GM_J = 0,       // column of the next iteration
  GM_DONE = 1,    // 1 once the residual estimate met the target or w vanished
  GM_BROKEN = 2,  // 1 when a non-finite norm appeared
  GM_TARGET = 3,  // absolute residual target
  GM_ITS = 4,     // iterations taken in this cycle
  GM_RES = 5,     // |g[j]| after the last iteration
  GM_INVWN = 6,   // 1 / ||w|| of the last iteration (0 when it vanished)
  GM_NRM2 = 7,    // ||w||^2 of the optional third projection pass
  GM_MISC = 16
};

struct GmView {
  double* part;
  int P, m;
  double *hcol, *h2, *cs, *sn, *g, *H, *y, *misc;
};

static size_t gm_doubles(int m) {
  const size_t P = (size_t)m + 2;
  return (size_t)kRedBlocks * P + 2 * P + 2 * (size_t)m + (m + 1) + (size_t)(m + 1) * m + m + GM_MISC;
}

static GmView gm_view(double* base, int m) {
  GmView G;
  G.P = m + 2;
  G.m = m;
  G.part = base;
  G.hcol = G.part + (size_t)kRedBlocks * G.P;
  G.h2 = G.hcol + G.P;
  G.cs = G.h2 + G.P;
  G.sn = G.cs + m;
  G.g = G.sn + m;
  G.H = G.g + (m + 1);
  G.y = G.H + (size_t)(m + 1) * m;
  G.misc = G.y + m;
  return G;
}

__device__ inline int gm_j(const GmView& G) { return (int)G.misc[GM_J]; }
__device__ inline bool gm_done(const GmView& G) { return G.misc[GM_DONE] != 0.0; }

// block sum of cnt <= MAXK values per thread into out[0 .. cnt) (same order
// as block_sum_store); ends with a barrier so that it can run in a loop
template <int MAXK>
__device__ inline void block_sum_row(double (&v)[MAXK], int cnt, double* out) {
  __shared__ double s[kRedThreads / 64][MAXK];
  const int lane = threadIdx.x % 64, wid = threadIdx.x / 64;
#pragma unroll
  for (int i = 0; i < MAXK; ++i) {
    if (i < cnt) {
      double x = v[i];
      for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
      if (lane == 0) s[wid][i] = x;
    }
  }
  __syncthreads();
  if ((int)threadIdx.x < cnt) {
    double t = 0;
    for (int w = 0; w < kRedThreads / 64; ++w) t += s[w][threadIdx.x];
    out[threadIdx.x] = t;
  }
  __syncthreads();
}

// partial dots of w with V_0 .. V_{K-1} and w . w (entry K), K = j + 1, in
// groups of kDotK entries
__global__ __launch_bounds__(kRedThreads) void k_gm_dots(GmView G, const double* __restrict__ V, long long n,
                                                         const double* __restrict__ w) {
  if (gm_done(G)) return;
  const int K = gm_j(G) + 1, cnt = K + 1;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (int g0 = 0; g0 < cnt; g0 += kDotK) {
    double acc[kDotK];
#pragma unroll
    for (int i = 0; i < kDotK; ++i) acc[i] = 0;
    for (long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += stride) {
      const double wr = w[r];
#pragma unroll
      for (int i = 0; i < kDotK; ++i) {
        const int ii = g0 + i;
        if (ii < K) acc[i] += V[(long long)ii * n + r] * wr;
        if (ii == K) acc[i] += wr * wr;
      }
    }
    block_sum_row<kDotK>(acc, cnt - g0 < kDotK ? cnt - g0 : kDotK, G.part + (size_t)blockIdx.x * G.P + g0);
  }
}

// w -= sum_i hcol_i V_i (i < K), then partial dots of the new w with V_0 ..
// V_{K-1} and w . w (entry K).  For K < kDotK one pass with the row of V in
// registers; otherwise the update first, then the dots in groups.
__global__ __launch_bounds__(kRedThreads) void k_gm_axpy_dots(GmView G, const double* __restrict__ V, long long n,
                                                              double* __restrict__ w) {
  if (gm_done(G)) return;
  const int K = gm_j(G) + 1, cnt = K + 1;
  const long long stride = (long long)gridDim.x * blockDim.x;
  const double* hc = G.hcol;
  if (K < kDotK) {
    double hh[kDotK], acc[kDotK];
#pragma unroll
    for (int i = 0; i < kDotK; ++i) {
      hh[i] = 0.0;
      if (i < K) hh[i] = hc[i];
      acc[i] = 0;
    }
    for (long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += stride) {
      double v[kDotK];
      double x = w[r];
#pragma unroll
      for (int i = 0; i < kDotK; ++i) {
        v[i] = 0.0;
        if (i < K) v[i] = V[(long long)i * n + r];
        x -= hh[i] * v[i];
      }
      w[r] = x;
#pragma unroll
      for (int i = 0; i < kDotK; ++i) {
        if (i < K) acc[i] += v[i] * x;
        if (i == K) acc[i] += x * x;
      }
    }
    block_sum_row<kDotK>(acc, cnt, G.part + (size_t)blockIdx.x * G.P);
    return;
  }
  for (long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += stride) {
    double x = w[r];
    for (int i = 0; i < K; ++i) x -= hc[i] * V[(long long)i * n + r];
    w[r] = x;
  }
  for (int g0 = 0; g0 < cnt; g0 += kDotK) {
    double acc[kDotK];
#pragma unroll
    for (int i = 0; i < kDotK; ++i) acc[i] = 0;
    for (long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += stride) {
      const double x = w[r];  // this thread's own rows, updated above
#pragma unroll
      for (int i = 0; i < kDotK; ++i) {
        const int ii = g0 + i;
        if (ii < K) acc[i] += V[(long long)ii * n + r] * x;
        if (ii == K) acc[i] += x * x;
      }
    }
    block_sum_row<kDotK>(acc, cnt - g0 < kDotK ? cnt - g0 : kDotK, G.part + (size_t)blockIdx.x * G.P + g0);
  }
}

// reorthogonalization (DGKS): when the projected norm dropped below 0.7 of
// the norm before the projection, w -= sum_i h2_i V_i and partial ||w||^2
__device__ inline bool gm_reorth(const GmView& G, int K) { return sqrt(G.h2[K]) < 0.7 * sqrt(G.hcol[K]); }

__global__ __launch_bounds__(kRedThreads) void k_gm_reorth(GmView G, const double* __restrict__ V, long long n,
                                                           double* __restrict__ w) {
  if (gm_done(G)) return;
  const int K = gm_j(G) + 1;
  if (!gm_reorth(G, K)) return;
  double acc[1] = {0};
  const long long stride = (long long)gridDim.x * blockDim.x;
  const double* hc = G.h2;
  if (K <= kDotK) {
    double hh[kDotK];
#pragma unroll
    for (int i = 0; i < kDotK; ++i) {
      hh[i] = 0.0;
      if (i < K) hh[i] = hc[i];
    }
    for (long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += stride) {
      double x = w[r];
#pragma unroll
      for (int i = 0; i < kDotK; ++i)
        if (i < K) x -= hh[i] * V[(long long)i * n + r];
      w[r] = x;
      acc[0] += x * x;
    }
  } else {
    for (long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += stride) {
      double x = w[r];
      for (int i = 0; i < K; ++i) x -= hc[i] * V[(long long)i * n + r];
      w[r] = x;
      acc[0] += x * x;
    }
  }
  block_sum_row<1>(acc, 1, G.part + (size_t)blockIdx.x * G.P);
}

// second stage of the reductions (fixed order, as k_reduce_parts): which 0:
// hcol[0 .. K], 1: h2[0 .. K], 2: the third pass's ||w||^2 (only when it ran)
__global__ void k_gm_reduce(GmView G, int which, int nblocks) {
  if (gm_done(G)) return;
  const int K = gm_j(G) + 1;
  if (which == 2 && !gm_reorth(G, K)) return;
  const int cnt = which == 2 ? 1 : K + 1;
  double* out = which == 0 ? G.hcol : which == 1 ? G.h2 : G.misc + GM_NRM2;
  __shared__ double s[256];
  for (int i = blockIdx.x; i < cnt; i += gridDim.x) {
    double t = 0;
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x) t += G.part[(long long)b * G.P + i];
    s[threadIdx.x] = t;
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
      if ((int)threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[i] = s[0];
    __syncthreads();
  }
}

// Hessenberg column, Givens rotations and the residual estimate of column j
// (one thread; products are not contracted, as on the host)
__global__ void k_gm_givens(GmView G) {
#pragma clang fp contract(off)
  if (threadIdx.x != 0 || blockIdx.x != 0 || gm_done(G)) return;
  const int j = gm_j(G), K = j + 1, m = G.m;
  double* hcol = G.hcol;
  double wn;
  if (gm_reorth(G, K)) {
    wn = sqrt(G.misc[GM_NRM2]);
    for (int i = 0; i < K; ++i) hcol[i] += G.h2[i];
  } else {
    wn = sqrt(G.h2[K]);
  }
  hcol[j + 1] = wn;
  if (!isfinite(wn)) {
    G.misc[GM_BROKEN] = 1.0;
    G.misc[GM_DONE] = 1.0;
    G.misc[GM_INVWN] = 0.0;
    return;
  }
  for (int i = 0; i < j; ++i) {
    const double a = G.cs[i] * hcol[i] + G.sn[i] * hcol[i + 1];
    const double b = -G.sn[i] * hcol[i] + G.cs[i] * hcol[i + 1];
    hcol[i] = a;
    hcol[i + 1] = b;
  }
  const double den = hypot(hcol[j], hcol[j + 1]);
  G.cs[j] = den > 0 ? hcol[j] / den : 1.0;
  G.sn[j] = den > 0 ? hcol[j + 1] / den : 0.0;
  hcol[j] = den;
  hcol[j + 1] = 0.0;
  G.g[j + 1] = -G.sn[j] * G.g[j];
  G.g[j] = G.cs[j] * G.g[j];
  for (int i = 0; i <= j; ++i) G.H[(size_t)i * m + j] = hcol[i];
  G.misc[GM_INVWN] = wn > 0 ? 1.0 / wn : 0.0;
  G.misc[GM_RES] = fabs(G.g[j + 1]);
  G.misc[GM_ITS] += 1.0;
  G.misc[GM_J] = (double)(j + 1);
  if (fabs(G.g[j + 1]) <= G.misc[GM_TARGET] || wn == 0) G.misc[GM_DONE] = 1.0;
}

// next basis vector V_{j+1} = w / ||w|| (j already advanced by k_gm_givens;
// skipped after a breakdown)
__global__ void k_gm_next(GmView G, double* __restrict__ V, long long n, const double* __restrict__ w) {
  if (G.misc[GM_BROKEN] != 0.0) return;
  const int j = gm_j(G);
  const double s = G.misc[GM_INVWN];
  double* vj = V + (long long)j * n;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) vj[i] = s * w[i];
}

// preconditioner input: V_j (cast to the preconditioner's precision)
template <typename To>
__global__ void k_gm_in(GmView G, const double* __restrict__ V, long long n, To* __restrict__ dst) {
  if (gm_done(G)) return;
  const double* vj = V + (long long)gm_j(G) * n;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = (To)vj[i];
}

// preconditioner output -> Z_j and the fixed FP64 input of the Jacobian
template <typename From>
__global__ void k_gm_out(GmView G, const From* __restrict__ src, long long n, double* __restrict__ Z,
                         double* __restrict__ zbuf) {
  if (gm_done(G)) return;
  double* zj = Z + (long long)gm_j(G) * n;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const double z = (double)src[i];
    zj[i] = z;
    zbuf[i] = z;
  }
}

// start of a cycle: V_0 = r / ||r||, g = (||r||, 0, ...), j = 0
__global__ void k_gm_start(GmView G, const double* __restrict__ r, double rnorm, double target, double* __restrict__ V,
                           long long n) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  const double s = 1.0 / rnorm;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) V[i] = s * r[i];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    for (int i = 0; i < GM_MISC; ++i) G.misc[i] = 0.0;
    G.misc[GM_TARGET] = target;
    G.misc[GM_RES] = rnorm;
    for (int i = 0; i <= G.m; ++i) G.g[i] = 0.0;
    G.g[0] = rnorm;
  }
}

// y = H^-1 g (upper triangular, jj columns), one thread, as on the host
__global__ void k_gm_backsub(GmView G, int jj) {
#pragma clang fp contract(off)
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int m = G.m;
  for (int i = jj - 1; i >= 0; --i) {
    double sum = G.g[i];
    for (int k2 = i + 1; k2 < jj; ++k2) sum -= G.H[(size_t)i * m + k2] * G.y[k2];
    G.y[i] = G.H[(size_t)i * m + i] != 0 ? sum / G.H[(size_t)i * m + i] : 0.0;
  }
}

static unsigned grid_for(long long n) {
  long long b = (n + 255) / 256;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  return (unsigned)b;
}

// the handle's diagonal in FP64 and FP32, computed once per linearization and
// kept until the next rotation or linearization (the volume and mortar terms
// are summed with atomics, so recomputing it may change its last bits)
int cached_diagonal(mns_handle* h, hipStream_t s) {
  const size_t n = (size_t)h->ndofs;
  hipError_t e;
  if (!h->d_diag64 && (e = hipMalloc((void**)&h->d_diag64, n * sizeof(double))) != hipSuccess)
    return set_error(h, MNS_ERR_HIP, std::string("hipMalloc: ") + hipGetErrorString(e));
  if (!h->d_diag32 && (e = hipMalloc((void**)&h->d_diag32, n * sizeof(float))) != hipSuccess)
    return set_error(h, MNS_ERR_HIP, std::string("hipMalloc: ") + hipGetErrorString(e));
  if (h->diag_valid) return MNS_OK;
  int rc = launch_diagonal<double>(h, h->d_diag64, s);
  if (rc) return rc;
  if ((rc = launch_cast_f64_f32(h->d_diag64, h->d_diag32, (int64_t)n, s))) return set_error(h, rc, "cast");
  h->diag_valid = true;
  return MNS_OK;
}

int launch_cast_f64_f32(const double* a, float* b, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL((k_cast<double, float>), dim3(grid_for(n)), dim3(256), 0, s, a, b, (long long)n);
  return hipGetLastError() == hipSuccess ? MNS_OK : MNS_ERR_HIP;
}

int launch_cast_f32_f64(const float* a, double* b, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL((k_cast<float, double>), dim3(grid_for(n)), dim3(256), 0, s, a, b, (long long)n);
  return hipGetLastError() == hipSuccess ? MNS_OK : MNS_ERR_HIP;
}

}  // namespace mns

using namespace mns;

namespace {

struct MG;
int mg_vcycle_body(MG* mg, const mns_solve_opts* o, hipStream_t s);
void* mg_io(MG* mg, bool out, bool f32);
void mg_count(MG* mg, int* v64, int* v32);

struct Solver {
  mns_handle* h;
  hipStream_t s;
  MG* mg = nullptr;
  long long n;
  int m;
  double *V, *Z, *w, *r, *t64a, *t64b;  // FP64 workspace
  float *b32, *x32, *r32, *d32, *t32;   // FP32 Chebyshev workspace
  double *b64c, *x64c, *r64c, *d64c;    // FP64 Chebyshev workspace
  int vm64 = 0, vm32 = 0;

  int err(int code, const std::string& msg) { return set_error(h, code, msg); }

  int sync_read(int K, double* host) {
    hipError_t e = hipMemcpyAsync(h->h_red, h->d_red + (size_t)kRedBlocks * 32, K * sizeof(double),
                                  hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return err(MNS_ERR_HIP, std::string("readback: ") + hipGetErrorString(e));
    std::memcpy(host, h->h_red, K * sizeof(double));
    return MNS_OK;
  }

  double* parts() { return h->d_red; }
  double* outs() { return h->d_red + (size_t)kRedBlocks * 32; }
  double* coefs() { return h->d_red + (size_t)kRedBlocks * 32 + 1024; }

  int reduce(int K) {
    hipLaunchKernelGGL(k_reduce_parts, dim3(K < 64 ? K : 64), dim3(256), 0, s, parts(), kRedBlocks, K, outs());
    return hipGetLastError() == hipSuccess ? MNS_OK : err(MNS_ERR_HIP, "reduce");
  }

  int jac64(const double* src, double* dst) {
    ++vm64;
    return launch_jacobian<double>(h, src, dst, s);
  }
  int jac32(const float* src, float* dst) {
    ++vm32;
    return launch_jacobian<float>(h, src, dst, s);
  }

  // Power iteration for the dominant eigenvalue magnitude of D^-1 J (FP64).
  // warm: t64a already holds a normalized iterate of an earlier estimate
  // (of a nearby operator), which is continued instead of restarting from 1
  int estimate_lambda(int iters, double* lam, bool warm = false) {
    int rc;
    double nrm = 0, val = 0;
    if (!warm) {
      // deterministic start vector: 1 on every DoF
      if ((rc = launch_fill<double>(t64a, 1.0, n, s))) return err(rc, "fill");
      nrm = std::sqrt((double)n);
      hipLaunchKernelGGL(k_scale_copy, dim3(grid_for(n)), dim3(256), 0, s, t64a, 1.0 / nrm, t64a, n);
    }
    for (int it = 0; it < iters; ++it) {
      if ((rc = jac64(t64a, t64b))) return rc;
      hipLaunchKernelGGL(k_power_step, dim3(kRedBlocks), dim3(kRedThreads), 0, s, t64b, h->d_diag64, t64a, n,
                         parts());
      if ((rc = reduce(1)) || (rc = sync_read(1, &val))) return rc;
      nrm = std::sqrt(val);
      if (!(nrm > 0) || !std::isfinite(nrm)) return err(MNS_ERR_HIP, "power iteration broke down");
      hipLaunchKernelGGL(k_scale_copy, dim3(grid_for(n)), dim3(256), 0, s, t64a, 1.0 / nrm, t64a, n);
    }
    *lam = nrm;
    return MNS_OK;
  }

  // z = Chebyshev(D^-1 J) approximation of J^-1 v, degree `deg`, interval [lmax/range, lmax]
  template <typename Real>
  int chebyshev(const Real* b, Real* x, Real* r, Real* d, Real* t, const Real* diag, int deg, double lmax,
                double range, const Real* sub = nullptr) {
    const double beta = lmax, alpha = lmax / range;
    const double theta = 0.5 * (beta + alpha), delta = 0.5 * (beta - alpha);
    const double sigma = theta / delta;
    double rho = 1.0 / sigma;
    const unsigned g = grid_for(n);
    hipLaunchKernelGGL(k_cheb_init<Real>, dim3(g), dim3(256), 0, s, b, diag, (Real)(1.0 / theta), r, d, x, n, sub);
    for (int k = 0; k < deg; ++k) {
      int rc;
      if constexpr (sizeof(Real) == 8) rc = jac64((const double*)d, (double*)t);
      else rc = jac32((const float*)d, (float*)t);
      if (rc) return rc;
      const double rho_new = 1.0 / (2.0 * sigma - rho);
      const double c1 = rho_new * rho, c2 = 2.0 * rho_new / delta;
      hipLaunchKernelGGL(k_cheb_step<Real>, dim3(g), dim3(256), 0, s, r, (const Real*)t, diag, (Real)c1, (Real)c2,
                         d, x, n);
      rho = rho_new;
    }
    return hipGetLastError() == hipSuccess ? MNS_OK : err(MNS_ERR_HIP, "chebyshev");
  }

  // One FGMRES iteration as a fixed sequence of launches: V_j (j read from
  // the device state) is copied or cast into the preconditioner's fixed input
  // buffer, the preconditioner body maps it to its fixed output buffer, which
  // is copied to Z_j and to the fixed input zbuf of the FP64 Jacobian, then
  // the Gram-Schmidt passes, the Givens update and the next basis vector.
  // No launch depends on j or on the host, so with use_graph the iteration
  // is captured once per solve and replayed.
  hipGraphExec_t gexec = nullptr;
  GmView G{};
  double* zbuf = nullptr;
  int it_vm64 = 0, it_vm32 = 0;  // Jacobian applications of one iteration

  int precond_body(const mns_solve_opts* o, double lmax, hipStream_t bs, int* v64, int* v32);

  int iteration(const mns_solve_opts* o, double lmax, hipStream_t st) {
    Solver B = *this;
    B.s = st;
    B.vm64 = B.vm32 = 0;
    const unsigned g = grid_for(n);
    const bool mgp = o->precond == MNS_PRECOND_MG || o->precond == MNS_PRECOND_MG64;
    const bool f32in = o->precond == MNS_F32 || o->precond == MNS_PRECOND_MG;
    void* in = mgp ? mg_io(mg, false, f32in) : (o->precond == MNS_F32 ? (void*)b32 : (void*)b64c);
    const void* out = mgp ? mg_io(mg, true, f32in)
                          : (o->precond == MNS_F32 ? (const void*)x32
                                                   : (o->precond == MNS_F64 ? (const void*)(d64c + n) : (const void*)b64c));
    if (f32in) hipLaunchKernelGGL(k_gm_in<float>, dim3(g), dim3(256), 0, st, G, V, n, (float*)in);
    else hipLaunchKernelGGL(k_gm_in<double>, dim3(g), dim3(256), 0, st, G, V, n, (double*)in);
    int rc;
    if (o->precond != -1 && (rc = precond_body(o, lmax, st, &B.vm64, &B.vm32))) return rc;
    if (f32in) hipLaunchKernelGGL(k_gm_out<float>, dim3(g), dim3(256), 0, st, G, (const float*)out, n, Z, zbuf);
    else hipLaunchKernelGGL(k_gm_out<double>, dim3(g), dim3(256), 0, st, G, (const double*)out, n, Z, zbuf);
    if ((rc = B.jac64(zbuf, w))) return rc;
    hipLaunchKernelGGL(k_gm_dots, dim3(kRedBlocks), dim3(kRedThreads), 0, st, G, (const double*)V, n, (const double*)w);
    hipLaunchKernelGGL(k_gm_reduce, dim3(64), dim3(256), 0, st, G, 0, kRedBlocks);
    hipLaunchKernelGGL(k_gm_axpy_dots, dim3(kRedBlocks), dim3(kRedThreads), 0, st, G, (const double*)V, n, w);
    hipLaunchKernelGGL(k_gm_reduce, dim3(64), dim3(256), 0, st, G, 1, kRedBlocks);
    hipLaunchKernelGGL(k_gm_reorth, dim3(kRedBlocks), dim3(kRedThreads), 0, st, G, (const double*)V, n, w);
    hipLaunchKernelGGL(k_gm_reduce, dim3(1), dim3(256), 0, st, G, 2, kRedBlocks);
    hipLaunchKernelGGL(k_gm_givens, dim3(1), dim3(64), 0, st, G);
    hipLaunchKernelGGL(k_gm_next, dim3(g), dim3(256), 0, st, G, V, n, (const double*)w);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return err(MNS_ERR_HIP, std::string("FGMRES iteration: ") + hipGetErrorString(e));
    it_vm64 = B.vm64;
    it_vm32 = B.vm32;
    return MNS_OK;
  }

  int capture_iteration(const mns_solve_opts* o, double lmax) {
    if (!h->cap && hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking) != hipSuccess)
      return err(MNS_ERR_HIP, "capture stream");
    hipError_t e = hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return err(MNS_ERR_HIP, std::string("begin capture: ") + hipGetErrorString(e));
    const int rc = iteration(o, lmax, h->cap);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(h->cap, &graph);
    if (rc) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc;
    }
    if (e != hipSuccess) return err(MNS_ERR_HIP, std::string("end capture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
      gexec = nullptr;
      return err(MNS_ERR_HIP, std::string("graph instantiate: ") + hipGetErrorString(e));
    }
    return MNS_OK;
  }

  void release_graph() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    gexec = nullptr;
  }

  // `count` iterations on the solver's stream (graph replays when enabled;
  // graphs need an untimed handle, since timed launches record events)
  int iterations(const mns_solve_opts* o, double lmax, int count) {
    int rc;
    if (o->use_graph && !h->timing_cap) {
      if (!gexec && (rc = capture_iteration(o, lmax))) return rc;
      for (int i = 0; i < count; ++i) {
        const hipError_t e = hipGraphLaunch(gexec, s);
        if (e != hipSuccess) return err(MNS_ERR_HIP, std::string("graph launch: ") + hipGetErrorString(e));
      }
      return MNS_OK;
    }
    for (int i = 0; i < count; ++i)
      if ((rc = iteration(o, lmax, s))) return rc;
    return MNS_OK;
  }

  // device state -> host (one synchronization)
  int read_state(double* misc) {
    hipError_t e = hipMemcpyAsync(h->h_red, G.misc, GM_MISC * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return err(MNS_ERR_HIP, std::string("readback: ") + hipGetErrorString(e));
    std::memcpy(misc, h->h_red, GM_MISC * sizeof(double));
    return MNS_OK;
  }

  // r = b - J x, returns ||r||
  int true_residual(const double* b, const double* x, double* rr, double* nrm) {
    int rc = jac64(x, rr);
    if (rc) return rc;
    hipLaunchKernelGGL(k_residual, dim3(kRedBlocks), dim3(kRedThreads), 0, s, b, rr, n, parts());
    double v;
    if ((rc = reduce(1)) || (rc = sync_read(1, &v))) return rc;
    *nrm = std::sqrt(v);
    return MNS_OK;
  }
};

// preconditioner body on stream bs: Chebyshev polynomial between the fixed
// buffers, or the V-cycle between level 0's vectors; adds its Jacobian
// applications to *v64 / *v32
int Solver::precond_body(const mns_solve_opts* o, double lmax, hipStream_t bs, int* v64, int* v32) {
  Solver B = *this;
  B.s = bs;
  B.vm64 = B.vm32 = 0;
  int rc;
  if (o->precond == MNS_PRECOND_MG || o->precond == MNS_PRECOND_MG64) {
    int a = 0, b = 0, c = 0, d = 0;
    mg_count(mg, &a, &b);
    rc = mg_vcycle_body(mg, o, bs);
    mg_count(mg, &c, &d);
    B.vm64 = c - a;
    B.vm32 = d - b;
  } else if (o->precond == MNS_F64) {
    rc = B.chebyshev<double>(b64c, d64c + n, r64c, d64c, t64b, h->d_diag64, o->cheb_degree, lmax, o->cheb_range);
  } else {
    rc = B.chebyshev<float>(b32, x32, r32, d32, t32, h->d_diag32, o->cheb_degree, lmax, o->cheb_range);
  }
  *v64 += B.vm64;
  *v32 += B.vm32;
  return rc;
}

int ensure_workspace(mns_handle* h, int m) {
  const size_t n = (size_t)h->ndofs;
  hipError_t e;
  if (h->ws_restart < m) {
    if (h->ws64) (void)hipFree(h->ws64);
    h->ws64 = nullptr;
    if ((e = hipMalloc((void**)&h->ws64, (size_t)(2 * m + 9) * n * sizeof(double))) != hipSuccess)
      return set_error(h, MNS_ERR_HIP, std::string("hipMalloc krylov: ") + hipGetErrorString(e));
    h->ws_restart = m;
    ++h->ws_gen;
  }
  if (!h->ws32 && (e = hipMalloc((void**)&h->ws32, 5 * n * sizeof(float))) != hipSuccess)
    return set_error(h, MNS_ERR_HIP, std::string("hipMalloc: ") + hipGetErrorString(e));
  if (!h->d_diag64 && (e = hipMalloc((void**)&h->d_diag64, n * sizeof(double))) != hipSuccess)
    return set_error(h, MNS_ERR_HIP, std::string("hipMalloc: ") + hipGetErrorString(e));
  if (!h->d_diag32 && (e = hipMalloc((void**)&h->d_diag32, n * sizeof(float))) != hipSuccess)
    return set_error(h, MNS_ERR_HIP, std::string("hipMalloc: ") + hipGetErrorString(e));
  if (h->gm_m < m) {
    if (h->d_gm) (void)hipFree(h->d_gm);
    h->d_gm = nullptr;
    h->gm_m = 0;
    if ((e = hipMalloc((void**)&h->d_gm, gm_doubles(m) * sizeof(double))) != hipSuccess)
      return set_error(h, MNS_ERR_HIP, std::string("hipMalloc FGMRES state: ") + hipGetErrorString(e));
    h->gm_m = m;
  }
  if (!h->d_red) {
    if ((e = hipMalloc((void**)&h->d_red, ((size_t)kRedBlocks * 32 + 2048) * sizeof(double))) != hipSuccess)
      return set_error(h, MNS_ERR_HIP, std::string("hipMalloc: ") + hipGetErrorString(e));
    if ((e = hipHostMalloc((void**)&h->h_red, 2048 * sizeof(double), hipHostMallocDefault)) != hipSuccess)
      return set_error(h, MNS_ERR_HIP, std::string("hipHostMalloc: ") + hipGetErrorString(e));
  }
  return MNS_OK;
}

// Solver view of a handle's workspace (restart m as allocated by
// ensure_workspace)
Solver make_solver(mns_handle* h, hipStream_t s, int m) {
  Solver S;
  S.h = h;
  S.s = s;
  S.n = h->ndofs;
  S.m = m;
  const size_t n = (size_t)h->ndofs;
  S.V = h->ws64;
  S.Z = h->ws64 + (size_t)(m + 1) * n;
  S.w = S.Z + (size_t)m * n;
  S.r = S.w + n;
  S.t64a = S.r + n;
  S.t64b = S.t64a + n;
  S.b64c = S.t64b + n;  // not used: the Chebyshev input is V_j itself
  S.r64c = S.b64c + n;
  S.d64c = S.r64c + n;
  S.x64c = nullptr;
  S.b32 = h->ws32;
  S.x32 = S.b32 + n;
  S.r32 = S.x32 + n;
  S.d32 = S.r32 + n;
  S.t32 = S.d32 + n;
  return S;
}

// ---------------------------------------------------------------------------
// Geometric multigrid on nested polar meshes (degree 2)
// ---------------------------------------------------------------------------

// 1D transfer tables of one direction between a fine and a coarse node line
// (degrees kf, kc; every coarse cell holds `refine` fine cells):
// prolongation rows (kc + 1 coarse nodes per fine node), restriction rows
// (the transposed entries, padded to a common width) and evaluation rows
// (kf + 1 fine nodes per coarse node: the fine field at the coarse nodes).
struct Tx1D {
  std::vector<int> pidx, ridx, eidx;
  std::vector<double> pw, rw, ew;
  int rwidth = 0;
};

static double snap(double w) {
  if (std::fabs(w) < 1e-13) return 0.0;
  if (std::fabs(w - 1.0) < 1e-13) return 1.0;
  return w;
}

static Tx1D build_tx1d(int kf, int kc, int ncc, int refine, bool periodic, const std::vector<double>& gf,
                       const std::vector<double>& gc, int rwidth) {
  Tx1D T;
  const int nfc = refine * ncc;
  const int nf = periodic ? kf * nfc : kf * nfc + 1;
  const int nc = periodic ? kc * ncc : kc * ncc + 1;
  const int PW = kc + 1, EW = kf + 1;
  T.pidx.assign((size_t)nf * PW, 0);
  T.pw.assign((size_t)nf * PW, 0.0);
  std::vector<std::vector<std::pair<int, double>>> rows(nc);
  std::vector<double> L(std::max(PW, EW)), dL(L.size()), d2L(L.size());
  for (int f = 0; f < nf; ++f) {
    int cf = f / kf, j = f % kf;
    if (cf == nfc) {  // last node of an open line
      cf = nfc - 1;
      j = kf;
    }
    const int c = cf / refine;
    const double xi = ((cf % refine) + gf[j]) / refine;
    lagrange_1d(gc, xi, L.data(), dL.data(), d2L.data());
    for (int a = 0; a < PW; ++a) {
      const double w = snap(L[a]);
      int idx = kc * c + a;
      if (periodic) idx %= nc;
      T.pidx[(size_t)f * PW + a] = idx;
      T.pw[(size_t)f * PW + a] = w;
      if (w != 0.0) rows[idx].push_back({f, w});
    }
  }
  for (auto& r : rows) T.rwidth = std::max(T.rwidth, (int)r.size());
  const int RW = std::max(rwidth, T.rwidth);
  T.ridx.assign((size_t)nc * RW, 0);
  T.rw.assign((size_t)nc * RW, 0.0);
  for (int c = 0; c < nc; ++c)
    for (size_t i = 0; i < rows[c].size(); ++i) {
      T.ridx[(size_t)c * RW + i] = rows[c][i].first;
      T.rw[(size_t)c * RW + i] = rows[c][i].second;
    }
  T.eidx.assign((size_t)nc * EW, 0);
  T.ew.assign((size_t)nc * EW, 0.0);
  for (int i = 0; i < nc; ++i) {
    int c = i / kc, a = i % kc;
    if (c == ncc) {
      c = ncc - 1;
      a = kc;
    }
    const double xc = gc[a] * refine;  // position in units of fine cells of coarse cell c
    int sub = (int)std::floor(xc);
    if (sub >= refine) sub = refine - 1;
    const int cf = c * refine + sub;
    lagrange_1d(gf, xc - sub, L.data(), dL.data(), d2L.data());
    for (int b = 0; b < EW; ++b) {
      int idx = kf * cf + b;
      if (periodic) idx %= nf;
      T.eidx[(size_t)i * EW + b] = idx;
      T.ew[(size_t)i * EW + b] = snap(L[b]);
    }
  }
  return T;
}

// device view of the transfer between level l (fine) and l + 1 (coarse)
struct TxView {
  int pw, rw, ew;               // row widths of the prolongation, restriction, evaluation tables
  int nc;                       // components
  int ntf, ntc, nzf, nzc;       // theta and z node counts (fine, coarse)
  int nrf[2], nrc[2];           // radial node rows per domain
  long long off1f, off1c;       // first stator node
  const int* idx;
  const double* w;
  long long pt, pr[2], pz, rt, rr[2], rz, et, er[2], ez;  // table offsets (entries)
};

// fine node g of P x_c (added to the fine value when add); entries flagged
// in mask (constrained rows, when given) receive a zero correction.  K1T, NCT:
// the row width and component count when known at compile time (coarse
// degree 2: 3; 4 components in 3D, 3 in 2D), so that the loops unroll and the
// components of a coarse node load together; 0: read from X
template <typename Real, int K1T = 0, int NCT = 0>
__device__ inline void prolong_node(const TxView& X, const Real* __restrict__ coarse, Real* __restrict__ fine,
                                    long long g, int add, const unsigned char* __restrict__ mask = nullptr) {
  const int dom = g >= X.off1f;
  const long long l = g - (dom ? X.off1f : 0);
  const int it = (int)(l % X.ntf);
  const long long l2 = l / X.ntf;
  const int nrf = dom ? X.nrf[1] : X.nrf[0];
  const int nrc = dom ? X.nrc[1] : X.nrc[0];
  const int ir = (int)(l2 % nrf), iz = (int)(l2 / nrf);
  const int K1 = K1T ? K1T : X.pw;
  const int NC = NCT ? NCT : X.nc;
  const long long ot = X.pt + (long long)it * K1, orr = (dom ? X.pr[1] : X.pr[0]) + (long long)ir * K1,
                  oz = X.pz + (long long)iz * K1;
  const long long cbase = dom ? X.off1c : 0;
  Real acc[4] = {0, 0, 0, 0};
#pragma unroll
  for (int a = 0; a < (K1T ? K1T : K1); ++a) {
    const double wt = X.w[ot + a];
    if (wt == 0.0) continue;
#pragma unroll
    for (int b = 0; b < (K1T ? K1T : K1); ++b) {
      const double wr = X.w[orr + b];
      if (wr == 0.0) continue;
#pragma unroll
      for (int c = 0; c < (K1T ? K1T : K1); ++c) {
        const double wz = X.w[oz + c];
        if (wz == 0.0) continue;
        const long long node = cbase + X.idx[ot + a] + (long long)X.ntc * (X.idx[orr + b] + (long long)nrc * X.idx[oz + c]);
        const Real ww = (Real)(wt * wr * wz);
#pragma unroll
        for (int m = 0; m < (NCT ? NCT : NC); ++m) acc[m] += ww * coarse[node * NC + m];
      }
    }
  }
#pragma unroll
  for (int m = 0; m < (NCT ? NCT : NC); ++m) {
    const Real c = (mask && mask[g * NC + m]) ? Real(0) : acc[m];
    fine[g * NC + m] = (add ? fine[g * NC + m] : Real(0)) + c;
  }
}

// the compile-time forms for coarse degree 2 (the coarse levels of every
// hierarchy here), else the general one
template <typename Real>
__device__ inline void prolong_node_any(const TxView& X, const Real* __restrict__ coarse, Real* __restrict__ fine,
                                        long long g, int add, const unsigned char* __restrict__ mask) {
  if (X.pw == 3 && X.nc == 4) prolong_node<Real, 3, 4>(X, coarse, fine, g, add, mask);
  else if (X.pw == 3 && X.nc == 3) prolong_node<Real, 3, 3>(X, coarse, fine, g, add, mask);
  else prolong_node<Real>(X, coarse, fine, g, add, mask);
}

template <typename Real>
__global__ void k_mg_prolong(TxView X, const Real* __restrict__ coarse, Real* __restrict__ fine, long long nnf,
                             int add, const unsigned char* __restrict__ mask) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < nnf) prolong_node_any(X, coarse, fine, g, add, mask);
}

// One direction of the restriction (the transposed 1D prolongation rows):
// the node grid of `in` has the coarse counts in the directions already
// restricted and the fine counts in the others; `out` has the coarse count in
// direction dir (0 theta, 1 r, 2 z).  Restricting theta, then r, then z reads
// each value a few times instead of once per coarse node of its support.
struct RestrictPass {
  int dir;
  int nt_in, nz_in, nr_in[2];
  int nt_out, nz_out, nr_out[2];
  long long off1_in, off1_out;  // first stator node of each grid
};

// output node g of one restriction pass
template <typename Real>
__device__ inline void restrict_dir_node(const TxView& X, const RestrictPass& P, const Real* __restrict__ in,
                                         Real* __restrict__ out, long long g,
                                         const unsigned char* __restrict__ mask = nullptr) {
  const int dom = g >= P.off1_out;
  const long long l = g - (dom ? P.off1_out : 0);
  const int it = (int)(l % P.nt_out);
  const long long l2 = l / P.nt_out;
  const int nro = dom ? P.nr_out[1] : P.nr_out[0];
  const int nri = dom ? P.nr_in[1] : P.nr_in[0];
  const int ir = (int)(l2 % nro), iz = (int)(l2 / nro);
  const int io = P.dir == 0 ? it : (P.dir == 1 ? ir : iz);
  const long long row = (P.dir == 0 ? X.rt : (P.dir == 1 ? (dom ? X.rr[1] : X.rr[0]) : X.rz)) + (long long)io * X.rw;
  const long long base = dom ? P.off1_in : 0;
  Real acc[4] = {0, 0, 0, 0};
  for (int a = 0; a < X.rw; ++a) {
    const double wa = X.w[row + a];
    if (wa == 0.0) continue;
    const int ii = X.idx[row + a];
    const int jt = P.dir == 0 ? ii : it, jr = P.dir == 1 ? ii : ir, jz = P.dir == 2 ? ii : iz;
    const long long node = base + jt + (long long)P.nt_in * (jr + (long long)nri * jz);
    for (int m = 0; m < X.nc; ++m) acc[m] += (Real)wa * in[node * X.nc + m];
  }
  for (int m = 0; m < X.nc; ++m) out[g * X.nc + m] = (mask && mask[g * X.nc + m]) ? Real(0) : acc[m];
}

// mask (last pass only): constrained entries of the coarse level set to zero
template <typename Real>
__global__ void k_mg_restrict_dir(TxView X, RestrictPass P, const Real* __restrict__ in, Real* __restrict__ out,
                                  long long nout, const unsigned char* __restrict__ mask) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < nout) restrict_dir_node(X, P, in, out, g, mask);
}


// coarse nodal values of a fine field: the fine field evaluated at the
// node counts of the two intermediate grids of the three-pass restriction
static long long restrict_tmp_nodes(const TxView& X) {
  return (long long)X.ntc * X.nzf * (X.nrf[0] + X.nrf[1] + X.nrc[0] + X.nrc[1]);
}

// the three passes of coarse = P^T fine (theta, then r, then z) and their
// output node counts; tmp holds the two intermediate grids, the second one
// n[0] * nc entries after the first
static void restrict_passes(const TxView& X, RestrictPass P[3], long long n[3]) {
  n[0] = (long long)X.ntc * X.nzf * (X.nrf[0] + X.nrf[1]);
  n[1] = (long long)X.ntc * X.nzf * (X.nrc[0] + X.nrc[1]);
  n[2] = (long long)X.ntc * X.nzc * (X.nrc[0] + X.nrc[1]);
  P[0] = RestrictPass{0, X.ntf, X.nzf, {X.nrf[0], X.nrf[1]}, X.ntc, X.nzf, {X.nrf[0], X.nrf[1]}, X.off1f,
                      (long long)X.ntc * X.nrf[0] * X.nzf};
  P[1] = RestrictPass{1, X.ntc, X.nzf, {X.nrf[0], X.nrf[1]}, X.ntc, X.nzf, {X.nrc[0], X.nrc[1]}, P[0].off1_out,
                      (long long)X.ntc * X.nrc[0] * X.nzf};
  P[2] = RestrictPass{2, X.ntc, X.nzf, {X.nrc[0], X.nrc[1]}, X.ntc, X.nzc, {X.nrc[0], X.nrc[1]}, P[1].off1_out,
                      X.off1c};
}

// coarse = P^T fine: theta, then r, then z (tmp holds the intermediate grids);
// cmask: constrained entries of the coarse level written as zero
template <typename Real>
static int mg_restrict(const TxView& X, void* tmp, const Real* fine, Real* coarse, hipStream_t s,
                       const unsigned char* cmask = nullptr) {
  RestrictPass P[3];
  long long n[3];
  restrict_passes(X, P, n);
  const long long n1 = n[0], n2 = n[1], n3 = n[2];
  const RestrictPass &p1 = P[0], &p2 = P[1], &p3 = P[2];
  Real* t1 = (Real*)tmp;
  Real* t2 = t1 + n1 * X.nc;
  hipLaunchKernelGGL(k_mg_restrict_dir<Real>, dim3((unsigned)((n1 + 255) / 256)), dim3(256), 0, s, X, p1, fine, t1, n1,
                     (const unsigned char*)nullptr);
  hipLaunchKernelGGL(k_mg_restrict_dir<Real>, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, s, X, p2,
                     (const Real*)t1, t2, n2, (const unsigned char*)nullptr);
  hipLaunchKernelGGL(k_mg_restrict_dir<Real>, dim3((unsigned)((n3 + 255) / 256)), dim3(256), 0, s, X, p3,
                     (const Real*)t2, coarse, n3, cmask);
  return hipGetLastError() == hipSuccess ? MNS_OK : MNS_ERR_HIP;
}

// coarse nodes (for nested degree-2 meshes a coarse node is a fine node)
__global__ void k_mg_eval(TxView X, const double* __restrict__ fine, double* __restrict__ coarse, long long nnc) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= nnc) return;
  const int dom = g >= X.off1c;
  const long long l = g - (dom ? X.off1c : 0);
  const int it = (int)(l % X.ntc);
  const long long l2 = l / X.ntc;
  const int nrf = dom ? X.nrf[1] : X.nrf[0];
  const int nrc = dom ? X.nrc[1] : X.nrc[0];
  const int ir = (int)(l2 % nrc), iz = (int)(l2 / nrc);
  const int KE = X.ew;
  const long long ot = X.et + (long long)it * KE, orr = (dom ? X.er[1] : X.er[0]) + (long long)ir * KE,
                  oz = X.ez + (long long)iz * KE;
  const long long fbase = dom ? X.off1f : 0;
  double acc[4] = {0, 0, 0, 0};
  for (int a = 0; a < KE; ++a) {
    const double wt = X.w[ot + a];
    if (wt == 0.0) continue;
    for (int b = 0; b < KE; ++b) {
      const double wr = X.w[orr + b];
      if (wr == 0.0) continue;
      for (int c = 0; c < KE; ++c) {
        const double wz = X.w[oz + c];
        if (wz == 0.0) continue;
        const long long node = fbase + X.idx[ot + a] + (long long)X.ntf * (X.idx[orr + b] + (long long)nrf * X.idx[oz + c]);
        const double ww = wt * wr * wz;
        for (int m = 0; m < X.nc; ++m) acc[m] += ww * fine[node * X.nc + m];
      }
    }
  }
  for (int m = 0; m < X.nc; ++m) coarse[g * X.nc + m] = acc[m];
}

__global__ void k_mask_clear(unsigned char* __restrict__ mask, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    mask[i] = 0;
}

__global__ void k_mask_set(const int64_t* __restrict__ cons, long long n, unsigned char* __restrict__ mask) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) mask[cons[i]] = 1;
}

// r = b - t with the constrained entries zero (the residual the cycle
// restricts; the same arithmetic as k_mg_axpy with beta = -1)
template <typename Real>
__global__ void k_mg_resid(const Real* __restrict__ b, const Real* __restrict__ t, Real* __restrict__ r,
                           const unsigned char* __restrict__ mask, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    r[i] = mask[i] ? Real(0) : b[i] + Real(-1) * t[i];
}

// out = a + beta * b
template <typename Real>
__global__ void k_mg_axpy(const Real* __restrict__ a, Real beta, const Real* __restrict__ b, Real* __restrict__ out,
                          long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    out[i] = a[i] + beta * b[i];
}

// restart length of a level's workspace: the caller's handle keeps its Krylov
// workspace, every other level (including a Picard copy of level 0) has
// restart 1, which holds the Chebyshev buffers
static int ws_of(mns_handle* hl, size_t l) { return (l == 0 && hl->ws_restart > 1) ? hl->ws_restart : 1; }

struct MGLevel {
  mns_handle* h = nullptr;  // level 0: the caller's handle (not owned)
  long long n = 0;
  void* b = nullptr;        // V-cycle vectors b, x, r (FP32 or FP64, room for FP64)
  double* inj = nullptr;    // injected state, history, force (coarse levels)
  void* tr = nullptr;       // intermediate grids of the three-pass restriction to the next level
  unsigned char* cmask = nullptr;  // 1 on the level's constrained entries (Dirichlet rows), else 0
  const double* eig_vec = nullptr;  // workspace vector holding the last power-iteration iterate
  const mns_handle* eig_h = nullptr; // handle whose operator it belongs to
  long long eig_gen = -1;           // workspace generation of that handle
  double lmax = 0;
};

struct MG {
  std::vector<MGLevel> L;
  std::vector<TxView> T;        // T[l]: level l <-> l + 1
  std::vector<void*> tables;    // device allocations of the tables
  long long version = -1;
  int max_levels = 0;           // level limit the hierarchy was built with
  int coarse_lin = -1;          // linearization kind of the coarse levels at the last setup
  int fine_lin = -1;            // and of the mesh's own level
  int eig_iters = -1;           // power iterations of the spectra at the last setup
  mns_handle* fine = nullptr;   // Picard copy of the mesh's own level (owned; level 0 when in use)
  int vm64 = 0, vm32 = 0;       // Jacobian applications launched by the cycles (all levels)
  void* coarse = nullptr;       // direct solve of the coarsest level (mns_coarse.hip)
  bool coarse_ready = false;    // it holds the inverse of the current coarsest operator
  int coarse_direct = -1;       // mg_coarse_direct at the last setup
};

// level 0's right-hand side b (out = false) or iterate x (out = true) in the
// cycle's precision (FP32 or FP64; the buffer holds room for FP64)
void* mg_io(MG* mg, bool out, bool f32) {
  MGLevel& L0 = mg->L[0];
  if (!out) return L0.b;
  return f32 ? (void*)((float*)L0.b + L0.n) : (void*)((double*)L0.b + L0.n);
}

void mg_count(MG* mg, int* v64, int* v32) {
  *v64 = mg->vm64;
  *v32 = mg->vm32;
}

// largest coarsest level solved directly (its dense matrix and inverse take
// 2 x 8 bytes x n^2: 1 GiB at this size)
constexpr int kCoarseDirectMax = 8192;

static int mg_err(mns_handle* h, hipError_t e, const char* what) {
  return set_error(h, MNS_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

static TxView make_tx(mns_handle* f, mns_handle* c, std::vector<void*>& keep, int* rc) {
  TxView X{};
  const int kf = f->k, kc = c->k;
  const int refine = f->desc.n_theta == c->desc.n_theta ? 1 : 2;
  X.nc = f->nc;
  X.ntf = f->ntn;
  X.ntc = c->ntn;
  X.nzf = f->nzn;
  X.nzc = c->nzn;
  for (int d = 0; d < 2; ++d) {
    X.nrf[d] = f->nrn[d];
    X.nrc[d] = c->nrn[d];
  }
  X.off1f = f->node_off1;
  X.off1c = c->node_off1;
  auto tx = [&](int ncc, bool periodic, int rwidth) {
    return build_tx1d(kf, kc, ncc, refine, periodic, f->gll, c->gll, rwidth);
  };
  // a first pass finds the widest restriction row of all directions
  int rw = 0;
  for (int pass = 0; pass < 2; ++pass) {
    Tx1D tt = tx(c->desc.n_theta, true, rw), tr0 = tx(c->desc.n_r_rotor, false, rw),
         tr1 = tx(c->desc.n_r_stator, false, rw);
    Tx1D tz;
    if (f->dim == 3) {
      tz = tx(c->desc.n_z, false, rw);
    } else {  // one node plane: identity
      tz.pidx.assign(kc + 1, 0);
      tz.pw.assign(kc + 1, 0.0);
      tz.pw[0] = 1.0;
      tz.eidx.assign(kf + 1, 0);
      tz.ew.assign(kf + 1, 0.0);
      tz.ew[0] = 1.0;
      tz.rwidth = 1;
      tz.ridx.assign(std::max(rw, 1), 0);
      tz.rw.assign(std::max(rw, 1), 0.0);
      tz.rw[0] = 1.0;
    }
    if (pass == 0) {
      rw = std::max(std::max(tt.rwidth, tr0.rwidth), std::max(tr1.rwidth, tz.rwidth));
      continue;
    }
    X.pw = kc + 1;
    X.rw = rw;
    X.ew = kf + 1;
    std::vector<int> idx;
    std::vector<double> w;
    auto put = [&](const std::vector<int>& i, const std::vector<double>& v) {
      const long long off = (long long)idx.size();
      idx.insert(idx.end(), i.begin(), i.end());
      w.insert(w.end(), v.begin(), v.end());
      return off;
    };
    X.pt = put(tt.pidx, tt.pw);
    X.pr[0] = put(tr0.pidx, tr0.pw);
    X.pr[1] = put(tr1.pidx, tr1.pw);
    X.pz = put(tz.pidx, tz.pw);
    X.rt = put(tt.ridx, tt.rw);
    X.rr[0] = put(tr0.ridx, tr0.rw);
    X.rr[1] = put(tr1.ridx, tr1.rw);
    X.rz = put(tz.ridx, tz.rw);
    X.et = put(tt.eidx, tt.ew);
    X.er[0] = put(tr0.eidx, tr0.ew);
    X.er[1] = put(tr1.eidx, tr1.ew);
    X.ez = put(tz.eidx, tz.ew);
    int* di = nullptr;
    double* dw = nullptr;
    hipError_t e;
    if ((e = hipMalloc((void**)&di, idx.size() * sizeof(int))) != hipSuccess ||
        (e = hipMalloc((void**)&dw, w.size() * sizeof(double))) != hipSuccess ||
        (e = hipMemcpy(di, idx.data(), idx.size() * sizeof(int), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(dw, w.data(), w.size() * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess) {
      *rc = mg_err(f, e, "multigrid tables");
    }
    keep.push_back(di);
    keep.push_back(dw);
    X.idx = di;
    X.w = dw;
  }
  return X;
}

static bool can_halve(const mns_mesh_desc& d) {
  const bool z = d.dim == 2 || d.n_z % 2 == 0;
  return d.n_theta % 2 == 0 && d.n_theta / 2 >= 4 && d.n_r_rotor % 2 == 0 && d.n_r_stator % 2 == 0 && z;
}

// Node positions of a coarse level of a curved (iso-parametric) hierarchy
// from those of the level above (host arrays, n_nodes x 3, the vector
// layout's node order): a halved degree-2 mesh takes every other node of the
// finer one (its cells are unions of 2^d finer cells, and the Q2 nodes of the
// union are finer nodes); the degree-2 level of a degree-3 mesh takes the Q3
// interpolant of each cell at the Q2 nodes.  Interface nodes are put at their
// polar positions on the circle, as the mortar requires (the Q3 interpolant
// of the circle deviates from it between the nodes).
static int iso_coarse_nodes(const mns_handle* hf, const std::vector<double>& xf, const mns_handle* hc,
                            std::vector<double>& xc) {
  const int dim = hc->desc.dim;
  const bool poly = hf->k == 3 && hc->k == 2;
  if (!poly && !(hf->k == 2 && hc->k == 2)) return MNS_ERR_UNSUPPORTED;
  // 1D rule per direction: coarse node index -> (fine indices, weights)
  double w3[4];  // Q3 Lagrange basis on its Gauss-Lobatto nodes at the cell midpoint
  {
    const double x[4] = {0.0, hf->gll[1], hf->gll[2], 1.0};
    for (int b = 0; b < 4; ++b) {
      double v = 1.0;
      for (int c = 0; c < 4; ++c)
        if (c != b) v *= (0.5 - x[c]) / (x[b] - x[c]);
      w3[b] = v;
    }
  }
  auto rule = [&](int j, int nfine, bool periodic, int* idx, double* w) {
    if (!poly) {
      idx[0] = 2 * j;
      w[0] = 1.0;
      return 1;
    }
    const int c = j / 2, a = j % 2;
    if (a == 0) {
      idx[0] = 3 * c;
      w[0] = 1.0;
      return 1;
    }
    for (int b = 0; b < 4; ++b) {
      idx[b] = periodic ? (3 * c + b) % nfine : 3 * c + b;
      w[b] = w3[b];
    }
    return 4;
  };
  xc.assign((size_t)hc->nnodes * 3, 0.0);
  for (int dom = 0; dom < 2; ++dom) {
    const long long fo = dom ? hf->node_off1 : 0, co = dom ? hc->node_off1 : 0;
    for (int iz = 0; iz < hc->nzn; ++iz) {
      int zi[4], ni_z = 1;
      double zw[4] = {1.0, 0, 0, 0};
      zi[0] = 0;
      if (dim == 3) ni_z = rule(iz, hf->nzn, false, zi, zw);
      for (int ir = 0; ir < hc->nrn[dom]; ++ir) {
        int ri[4];
        double rw[4];
        const int ni_r = rule(ir, hf->nrn[dom], false, ri, rw);
        for (int it = 0; it < hc->ntd[dom]; ++it) {
          int ti[4];
          double tw[4];
          const int ni_t = rule(it, hf->ntd[dom], true, ti, tw);
          double p[3] = {0, 0, 0};
          for (int c = 0; c < ni_z; ++c)
            for (int b = 0; b < ni_r; ++b)
              for (int a = 0; a < ni_t; ++a) {
                const long long nd = fo + ti[a] + (long long)hf->ntd[dom] * (ri[b] + (long long)hf->nrn[dom] * zi[c]);
                const double ww = zw[c] * rw[b] * tw[a];
                for (int m = 0; m < 3; ++m) p[m] += ww * xf[(size_t)nd * 3 + m];
              }
          const long long cn = co + it + (long long)hc->ntd[dom] * (ir + (long long)hc->nrn[dom] * iz);
          const bool iface = dom == 0 ? ir == hc->nrn[0] - 1 : ir == 0;
          if (iface) {
            const double th = (it / hc->k + hc->gll[it % hc->k]) * hc->dthd[dom];
            p[0] = hc->desc.r_interface * std::cos(th);
            p[1] = hc->desc.r_interface * std::sin(th);
            p[2] = dim == 3 ? (iz / hc->k + hc->gll[iz % hc->k]) * hc->dz : 0.0;
          }
          for (int m = 0; m < 3; ++m) xc[(size_t)cn * 3 + m] = p[m];
        }
      }
    }
  }
  return MNS_OK;
}

// the handle's node positions (curved meshes), device -> host
static int iso_host_nodes(mns_handle* h, std::vector<double>& x) {
  x.resize((size_t)h->nnodes * 3);
  const hipError_t e = hipMemcpy(x.data(), h->d_xnode, x.size() * sizeof(double), hipMemcpyDeviceToHost);
  return e == hipSuccess ? MNS_OK : set_error(h, MNS_ERR_HIP, std::string("node positions: ") + hipGetErrorString(e));
}

// levels and tables (once per handle)
static int mg_build(mns_handle* h, int max_levels, MG** out) {
  if (h->mg) {
    MG* old = (MG*)h->mg;
    if (old->max_levels == max_levels) {
      *out = old;
      return MNS_OK;
    }
    mg_free(h);  // another level count was asked for
  }
  if (h->k != 2 && h->k != 3) return set_error(h, MNS_ERR_UNSUPPORTED, "multigrid needs degree 2 or 3");
  if (!h->equal_rings) return set_error(h, MNS_ERR_UNSUPPORTED, "multigrid needs equal interface cell counts");
  MG* mg = new MG();
  mg->max_levels = max_levels;
  h->mg = mg;
  MGLevel L0;
  L0.h = h;
  L0.n = h->ndofs;
  mg->L.push_back(L0);
  mns_mesh_desc d = h->desc;
  d.n_theta_stator = 0;  // equal ring counts on every level
  // curved meshes: every coarse level gets node positions from the level above
  std::vector<double> xprev, xcur;
  if (h->iso) {
    int rc = iso_host_nodes(h, xprev);
    if (rc) return rc;
  }
  // degree 3: first a degree-2 level on the same mesh, then halved meshes
  bool poly = d.degree == 3;
  while ((poly || can_halve(d)) && (max_levels == 0 || (int)mg->L.size() < max_levels)) {
    if (poly) {
      d.degree = 2;
      poly = false;
    } else {
      d.n_theta /= 2;
      d.n_r_rotor /= 2;
      d.n_r_stator /= 2;
      if (d.dim == 3) d.n_z /= 2;
    }
    mns_handle* hc = new mns_handle();
    int rc = mns_build_handle(&d, h->stream, hc);
    if (!rc && h->iso) {
      rc = iso_coarse_nodes(mg->L.back().h, xprev, hc, xcur);
      if (!rc) rc = iso_set_nodes(hc, xcur.data(), hc->nnodes, h->stream);
      xprev.swap(xcur);
    }
    if (rc) {
      const std::string msg = hc->err;
      mns_destroy(hc);
      return set_error(h, rc, "multigrid level: " + msg);
    }
    MGLevel Lc;
    Lc.h = hc;
    Lc.n = hc->ndofs;
    mg->L.push_back(Lc);
  }
  int rc = MNS_OK;
  for (size_t l = 0; l + 1 < mg->L.size(); ++l) {
    mg->T.push_back(make_tx(mg->L[l].h, mg->L[l + 1].h, mg->tables, &rc));
    if (rc) return rc;
  }
  hipError_t e;
  for (size_t l = 0; l < mg->L.size(); ++l) {
    MGLevel& Lv = mg->L[l];
    if ((e = hipMalloc(&Lv.b, 3 * (size_t)Lv.n * sizeof(double))) != hipSuccess) return mg_err(h, e, "hipMalloc mg");
    if (l > 0 && (e = hipMalloc((void**)&Lv.inj, 3 * (size_t)Lv.n * sizeof(double))) != hipSuccess)
      return mg_err(h, e, "hipMalloc mg");
    if (l + 1 < mg->L.size() &&
        (e = hipMalloc(&Lv.tr, (size_t)restrict_tmp_nodes(mg->T[l]) * Lv.h->nc * sizeof(double))) != hipSuccess)
      return mg_err(h, e, "hipMalloc mg");
    // constrained-entry mask of the level (the constraint list is fixed by
    // the mesh): the cycle zeroes these entries inside its fused kernels
    if ((e = hipMalloc((void**)&Lv.cmask, (size_t)Lv.n)) != hipSuccess) return mg_err(h, e, "hipMalloc mg");
    hipLaunchKernelGGL(k_mask_clear, dim3(grid_for(Lv.n)), dim3(256), 0, h->stream, Lv.cmask, Lv.n);
    if (Lv.h->n_cons > 0)
      hipLaunchKernelGGL(k_mask_set, dim3((unsigned)((Lv.h->n_cons + 255) / 256)), dim3(256), 0, h->stream,
                         (const int64_t*)Lv.h->d_cons, (long long)Lv.h->n_cons, Lv.cmask);
  }
  if ((e = hipStreamSynchronize(h->stream)) != hipSuccess) return mg_err(h, e, "multigrid masks");
  *out = mg;
  return MNS_OK;
}

// coarse operators at the current angle and state, diagonals and spectra
static int mg_setup(mns_handle* h, MG* mg, const mns_solve_opts* o, hipStream_t s) {
  if (mg->version == h->lin_version && mg->coarse_lin == o->mg_coarse_linearization &&
      mg->fine_lin == o->mg_fine_linearization && mg->eig_iters == o->eig_iters &&
      mg->coarse_direct == o->mg_coarse_direct)
    return MNS_OK;
  int rc;
  // level 0: the caller's handle, or a copy of its mesh with the Picard
  // linearization at the same state (the outer FGMRES keeps the caller's)
  if (o->mg_fine_linearization == MNS_LIN_PICARD) {
    if (!mg->fine) {
      mns_handle* hf = new mns_handle();
      std::vector<double> xf;
      if (!(rc = mns_build_handle(&h->desc, h->stream, hf)) && h->iso && !(rc = iso_host_nodes(h, xf)))
        rc = iso_set_nodes(hf, xf.data(), hf->nnodes, s);
      if (rc) {
        const std::string msg = hf->err.empty() ? h->err : hf->err;
        mns_destroy(hf);
        return set_error(h, rc, "multigrid fine copy: " + msg);
      }
      mg->fine = hf;
    }
    mns_handle* hf = mg->fine;
    hf->fused = h->fused;
    hf->quad = h->quad;
    if ((rc = mns_rotate_rotor(hf, h->theta, h->omega, s))) return set_error(h, rc, "fine copy rotate: " + hf->err);
    hf->picard = 1;
    if ((rc = mns_set_linearization(hf, h->d_state, h->d_hist, h->d_force, s)))
      return set_error(h, rc, "fine copy linearization: " + hf->err);
    mg->L[0].h = hf;
  } else {
    mg->L[0].h = h;
  }
  for (size_t l = 1; l < mg->L.size(); ++l) {
    MGLevel& Lv = mg->L[l];
    mns_handle* hc = Lv.h;
    mns_handle* hf = mg->L[l - 1].h;
    const TxView& X = mg->T[l - 1];
    const long long nnc = hc->nnodes;
    const unsigned g = (unsigned)((nnc + 255) / 256);
    const double* fsrc[3] = {hf->d_state, hf->d_hist, hf->d_force};
    double* cdst[3] = {Lv.inj, Lv.inj + Lv.n, Lv.inj + 2 * Lv.n};
    for (int i = 0; i < 3; ++i)
      if (fsrc[i]) hipLaunchKernelGGL(k_mg_eval, dim3(g), dim3(256), 0, s, X, fsrc[i], cdst[i], nnc);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return mg_err(h, e, "injection");
    if ((rc = mns_rotate_rotor(hc, h->theta, h->omega, s))) return set_error(h, rc, "coarse rotate: " + hc->err);
    hc->picard = o->mg_coarse_linearization == MNS_LIN_PICARD;
    if ((rc = mns_set_linearization(hc, cdst[0], fsrc[1] ? cdst[1] : nullptr, fsrc[2] ? cdst[2] : nullptr, s)))
      return set_error(h, rc, "coarse linearization: " + hc->err);
  }
  for (size_t l = 0; l < mg->L.size(); ++l) {
    MGLevel& Lv = mg->L[l];
    mns_handle* hl = Lv.h;
    if ((rc = ensure_workspace(hl, ws_of(hl, l)))) return l ? set_error(h, rc, hl->err) : rc;
    if (!hl->diag_valid) {
      if ((rc = launch_diagonal<double>(hl, hl->d_diag64, s))) return set_error(h, rc, "diagonal: " + hl->err);
      if ((rc = launch_cast_f64_f32(hl->d_diag64, hl->d_diag32, (int64_t)hl->ndofs, s))) return set_error(h, rc, "cast");
      hl->diag_valid = true;
    }
    Solver S = make_solver(hl, s, ws_of(hl, l));
    // spectra after a relinearization or rotation: continue the previous
    // power iteration of the level (same workspace) for a quarter of the
    // iterations; a first setup starts from the constant vector
    const bool warm = Lv.eig_vec == S.t64a && Lv.eig_h == hl && Lv.eig_gen == hl->ws_gen;
    const int iters = warm ? std::max(4, o->eig_iters / 4) : o->eig_iters;
    if ((rc = S.estimate_lambda(iters, &Lv.lmax, warm))) return l ? set_error(h, rc, hl->err) : rc;
    Lv.eig_vec = S.t64a;
    Lv.eig_h = hl;
    Lv.eig_gen = hl->ws_gen;
  }
  // coarsest level of a hierarchy of two or more levels: its matrix,
  // reconstructed and inverted in FP64 (too large a level keeps the FP64
  // Chebyshev polynomial)
  mg->coarse_ready = false;
  if (o->mg_coarse_direct && mg->L.size() >= 2) {
    mns_handle* hc = mg->L.back().h;
    rc = coarse_setup(hc, &mg->coarse, s, kCoarseDirectMax);
    if (rc == MNS_OK) mg->coarse_ready = true;
    else if (rc != MNS_ERR_UNSUPPORTED) return set_error(h, rc, "coarse direct solve: " + hc->err);
  }
  mg->coarse_direct = o->mg_coarse_direct;
  mg->version = h->lin_version;
  mg->coarse_lin = o->mg_coarse_linearization;
  mg->fine_lin = o->mg_fine_linearization;
  mg->eig_iters = o->eig_iters;
  return MNS_OK;
}

// x = Chebyshev smoothing of J x = b at level l (from x = 0 when zero)
// FP32 or FP64 views of a level's work vectors and its Chebyshev buffers
template <typename Real>
struct MGVec {
  Real *b, *x, *r;           // V-cycle vectors of the level
  Real *cr, *cd, *ct, *cx;   // Chebyshev buffers of the level's solver workspace
  const Real* diag;
};

template <typename Real>
static MGVec<Real> mg_vec(MGLevel& Lv, const Solver& S) {
  MGVec<Real> v;
  Real* base = (Real*)Lv.b;
  v.b = base;
  v.x = base + Lv.n;
  v.r = base + 2 * Lv.n;
  if constexpr (sizeof(Real) == 4) {
    v.cr = S.r32;
    v.cd = S.d32;
    v.ct = S.t32;
    v.cx = S.x32;
    v.diag = Lv.h->d_diag32;
  } else {
    v.cr = S.r64c;
    v.cd = S.d64c;
    v.ct = S.t64b;
    v.cx = S.d64c + Lv.n;  // the spare vector after the Chebyshev buffers
    v.diag = Lv.h->d_diag64;
  }
  return v;
}

// x = Chebyshev smoothing of J x = b at level l (from x = 0 when zero)
template <typename Real>
static int mg_smooth(MG* mg, size_t l, const Real* b, Real* x, bool zero, int deg, double range, double fac,
                     hipStream_t s) {
  MGLevel& Lv = mg->L[l];
  const double lmax = fac * Lv.lmax;
  mns_handle* hl = Lv.h;
  Solver S = make_solver(hl, s, ws_of(hl, l));
  MGVec<Real> v = mg_vec<Real>(Lv, S);
  const unsigned g = grid_for(Lv.n);
  int& count = sizeof(Real) == 8 ? mg->vm64 : mg->vm32;
  if (zero) {
    const int rc = S.chebyshev<Real>(b, x, v.cr, v.cd, v.ct, v.diag, deg, lmax, range);
    count += S.vm64 + S.vm32;
    return rc;
  }
  // x += poly(b - J x): the residual is formed by the polynomial's first kernel
  int rc = launch_jacobian<Real>(hl, x, v.r, s);
  if (rc) return rc;
  ++count;
  rc = S.chebyshev<Real>(b, v.cx, v.cr, v.cd, v.ct, v.diag, deg, lmax, range, (const Real*)v.r);
  count += S.vm64 + S.vm32;
  if (rc) return rc;
  hipLaunchKernelGGL(k_mg_axpy<Real>, dim3(g), dim3(256), 0, s, (const Real*)x, Real(1), (const Real*)v.cx, x, Lv.n);
  return hipGetLastError() == hipSuccess ? MNS_OK : MNS_ERR_HIP;
}

// coarsest-level solve in FP64 for an FP32 cycle: b (FP32) -> FP64, Chebyshev
// of degree mg_coarse_degree with FP64 Jacobian applications, x (FP32) <- FP64
static int mg_coarse_f64(MG* mg, size_t l, const float* b, float* x, const mns_solve_opts* o, hipStream_t s) {
  MGLevel& Lv = mg->L[l];
  mns_handle* hl = Lv.h;
  Solver S = make_solver(hl, s, ws_of(hl, l));
  const unsigned g = grid_for(Lv.n);
  hipLaunchKernelGGL((k_cast<float, double>), dim3(g), dim3(256), 0, s, b, S.w, (long long)Lv.n);
  const double lmax = o->cheb_lambda_factor * Lv.lmax;
  int rc = S.chebyshev<double>(S.w, S.r, S.r64c, S.d64c, S.t64b, hl->d_diag64, o->mg_coarse_degree, lmax,
                               o->mg_smooth_range);
  mg->vm64 += S.vm64;
  if (rc) return rc;
  hipLaunchKernelGGL((k_cast<double, float>), dim3(g), dim3(256), 0, s, (const double*)S.r, x, (long long)Lv.n);
  return hipGetLastError() == hipSuccess ? MNS_OK : MNS_ERR_HIP;
}

template <typename Real>
static int mg_cycle(MG* mg, size_t l, const mns_solve_opts* o, hipStream_t s) {
  MGLevel& Lv = mg->L[l];
  mns_handle* hl = Lv.h;
  Solver S = make_solver(hl, s, ws_of(hl, l));
  MGVec<Real> v = mg_vec<Real>(Lv, S);
  int rc;
  if (l + 1 == mg->L.size()) {
    // coarsest level: in FP64 whatever the smoothers' precision (the FP32
    // right-hand side is widened into the level's FP64 work vectors w, r,
    // which no coarse level otherwise uses, and the result narrowed back);
    // a hierarchy of one level keeps the smoothers' precision
    if (mg->coarse_ready && l > 0) {
      const int rc2 = coarse_apply<Real>(mg->coarse, v.b, v.x, s);
      return rc2 ? set_error(mg->L[0].h, rc2, "coarse direct solve") : MNS_OK;
    }
    if (sizeof(Real) == 4 && l > 0) return mg_coarse_f64(mg, l, (const float*)v.b, (float*)v.x, o, s);
    return mg_smooth<Real>(mg, l, v.b, v.x, true, o->mg_coarse_degree, o->mg_smooth_range, o->cheb_lambda_factor, s);
  }
  if ((rc = mg_smooth<Real>(mg, l, v.b, v.x, true, o->mg_smooth_degree, o->mg_smooth_range, o->cheb_lambda_factor,
                            s)))
    return rc;
  // residual, restricted with constrained rows zero on both levels
  if ((rc = launch_jacobian<Real>(hl, v.x, v.ct, s))) return rc;
  ++(sizeof(Real) == 8 ? mg->vm64 : mg->vm32);
  const unsigned g = grid_for(Lv.n);
  hipLaunchKernelGGL(k_mg_resid<Real>, dim3(g), dim3(256), 0, s, (const Real*)v.b, (const Real*)v.ct, v.r,
                     (const unsigned char*)Lv.cmask, Lv.n);
  MGLevel& Lc = mg->L[l + 1];
  Solver Sc = make_solver(Lc.h, s, 1);
  MGVec<Real> vc = mg_vec<Real>(Lc, Sc);
  const TxView& X = mg->T[l];
  if ((rc = mg_restrict<Real>(X, Lv.tr, (const Real*)v.r, vc.b, s, Lc.cmask)))
    return set_error(mg->L[0].h, rc, "multigrid restriction");
  if ((rc = mg_cycle<Real>(mg, l + 1, o, s))) return rc;
  // x += P x_c (constrained rows of the correction zero)
  hipLaunchKernelGGL(k_mg_prolong<Real>, dim3((unsigned)((hl->nnodes + 255) / 256)), dim3(256), 0, s, X,
                     (const Real*)vc.x, v.x, (long long)hl->nnodes, 1, (const unsigned char*)Lv.cmask);
  if (hipGetLastError() != hipSuccess) return set_error(mg->L[0].h, MNS_ERR_HIP, "multigrid kernels");
  return mg_smooth<Real>(mg, l, v.b, v.x, false, o->mg_smooth_degree, o->mg_smooth_range, o->cheb_lambda_factor, s);
}

int mg_vcycle_body(MG* mg, const mns_solve_opts* o, hipStream_t s) {
  return o->precond == MNS_PRECOND_MG64 ? mg_cycle<double>(mg, 0, o, s) : mg_cycle<float>(mg, 0, o, s);
}

}  // namespace

// ---------------------------------------------------------------------------
// Multigrid of one instance inside a batched solve (mns_batch_solver.hip):
// the finest level's smoothing runs batched over the instances; the
// coarse-grid correction runs per instance through the code above.
// ---------------------------------------------------------------------------
namespace mns {

int mg_instance_setup(mns_handle* h, const mns_solve_opts* o, hipStream_t s, mns_handle** level0, double* lmax0) {
  int rc = ensure_workspace(h, 1);
  if (rc) return rc;
  MG* mg = nullptr;
  if ((rc = mg_build(h, o->mg_levels, &mg))) return rc;
  // one level would make the cycle a plain polynomial, not smoothing plus
  // a coarse-grid correction
  if (mg->L.size() < 2)
    return set_error(h, MNS_ERR_UNSUPPORTED,
                     "batched multigrid needs two or more levels (degree 3, or a mesh that can be halved)");
  if ((rc = mg_setup(h, mg, o, s))) return rc;
  *level0 = mg->L[0].h;
  *lmax0 = mg->L[0].lmax;
  return MNS_OK;
}

template <typename Real>
int mg_instance_correction(mns_handle* h, const Real* r0, Real* x0, const mns_solve_opts* o, hipStream_t s) {
  MG* mg = (MG*)h->mg;
  if (!mg || mg->L.size() < 2) return set_error(h, MNS_ERR_INVALID_ARG, "multigrid hierarchy missing");
  MGLevel& L0 = mg->L[0];
  mns_handle* h0 = L0.h;
  MGLevel& Lc = mg->L[1];
  Solver Sc = make_solver(Lc.h, s, 1);
  MGVec<Real> vc = mg_vec<Real>(Lc, Sc);
  const TxView& X = mg->T[0];
  int rc;
  if ((rc = mg_restrict<Real>(X, L0.tr, r0, vc.b, s, Lc.cmask))) return set_error(h, rc, "multigrid restriction");
  if ((rc = mg_cycle<Real>(mg, 1, o, s))) return rc;
  hipLaunchKernelGGL(k_mg_prolong<Real>, dim3((unsigned)((h0->nnodes + 255) / 256)), dim3(256), 0, s, X,
                     (const Real*)vc.x, x0, (long long)h0->nnodes, 1, (const unsigned char*)L0.cmask);
  return hipGetLastError() == hipSuccess ? MNS_OK : set_error(h, MNS_ERR_HIP, "multigrid correction kernels");
}
template int mg_instance_correction<float>(mns_handle*, const float*, float*, const mns_solve_opts*, hipStream_t);
template int mg_instance_correction<double>(mns_handle*, const double*, double*, const mns_solve_opts*, hipStream_t);

void mg_instance_counts(mns_handle* h, int* v64, int* v32) {
  MG* mg = (MG*)h->mg;
  *v64 = *v32 = 0;
  if (mg) mg_count(mg, v64, v32);
}

}  // namespace mns

// ---------------------------------------------------------------------------
// The coarse-grid correction of every instance of a batch at once.  Level l
// holds the instances whose hierarchy reaches it, the deepest first, so that
// those with a coarser level below form a prefix: their smoothing runs as
// batch launches over their level-l operators (per-instance lambda_max and
// diagonal), the others take their direct FP64 coarsest solve in one batched
// launch.  Restriction, prolongation and constraints run as item launches
// (one item per instance, blocks in item order), with each instance's own
// transfer tables.  The steps are those of the single-instance cycle.
// ---------------------------------------------------------------------------
namespace {

struct TxItem {
  TxView X;
  RestrictPass P[3];
  long long n[3];        // output nodes of the restriction passes
  long long blk[4];      // first block in the launches of passes 0..2 and of the prolongation
  long long nnf;         // fine nodes (prolongation outputs)
  void* tmp;             // intermediate grids of the restriction (the instance's own buffer)
  long long foff, coff;  // the instance's first entry in the fine and in the coarse level vectors
};

struct ConsItem {
  const int64_t* cons;  // constrained rows of the instance's level (sorted)
  long long n;
  long long off;        // the instance's first entry in the level vector
  long long blk0;
};

// last item whose first block of launch `which` is at or before block b
template <typename Item, typename Get>
__device__ inline int item_find(const Item* it, int count, long long b, Get first) {
  int a = 0, z = count - 1;
  while (a < z) {
    const int mid = (a + z + 1) >> 1;
    if (first(it[mid]) <= b) a = mid;
    else z = mid - 1;
  }
  return a;
}

// restriction pass `pass` of every item: pass 0 reads the fine level vector,
// pass 2 writes the coarse one
template <typename Real>
__global__ __launch_bounds__(256) void k_bmg_restrict(const TxItem* __restrict__ items, int count, int pass,
                                                      const Real* __restrict__ fine, Real* __restrict__ coarse) {
  const TxItem& it = items[item_find(items, count, blockIdx.x, [pass](const TxItem& t) { return t.blk[pass]; })];
  const long long g = ((long long)blockIdx.x - it.blk[pass]) * 256 + threadIdx.x;
  if (g >= it.n[pass]) return;
  Real* t1 = (Real*)it.tmp;
  Real* t2 = t1 + it.n[0] * it.X.nc;
  const Real* in = pass == 0 ? fine + it.foff : (pass == 1 ? t1 : t2);
  Real* out = pass == 0 ? t1 : (pass == 1 ? t2 : coarse + it.coff);
  restrict_dir_node(it.X, it.P[pass], in, out, g);
}

template <typename Real>
__global__ __launch_bounds__(256) void k_bmg_prolong(const TxItem* __restrict__ items, int count,
                                                     const Real* __restrict__ coarse, Real* __restrict__ fine) {
  const TxItem& it = items[item_find(items, count, blockIdx.x, [](const TxItem& t) { return t.blk[3]; })];
  const long long g = ((long long)blockIdx.x - it.blk[3]) * 256 + threadIdx.x;
  if (g < it.nnf) prolong_node_any(it.X, coarse + it.coff, fine + it.foff, g, 0, (const unsigned char*)nullptr);
}

// constrained rows of every item set to zero
template <typename Real>
__global__ __launch_bounds__(256) void k_bmg_constraints(const ConsItem* __restrict__ items, int count,
                                                         Real* __restrict__ v) {
  const ConsItem& it = items[item_find(items, count, blockIdx.x, [](const ConsItem& t) { return t.blk0; })];
  const long long i = ((long long)blockIdx.x - it.blk0) * 256 + threadIdx.x;
  if (i < it.n) v[it.off + it.cons[i]] = Real(0);
}

// Chebyshev scalars of count instances from their lambda_max
__global__ void k_bmg_coef(const double* __restrict__ lam, int count, int deg, double lambda_factor, double range,
                           double* inv_theta, double* cheb) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x)
    cheb_scalars(lam[i], lambda_factor, range, deg, count, i, inv_theta, cheb);
}

}  // namespace

namespace mns {

struct BatchMG {
  struct Level {
    int count = 0, ncont = 0;        // instances on the level; those with a coarser level (a prefix)
    long long n = 0, ncn = 0;        // entries of all of them; of the prefix
    std::vector<long long> off;      // first entry of each (count + 1)
    mns_batch* bat = nullptr;        // batch over the prefix's level operators (levels >= 1)
    long long* d_seg = nullptr;      // segments of the prefix: first blocks, first entries (ncont + 1 each)
    long long nblk = 0;              // vector blocks of the prefix
    double* d_coef = nullptr;        // inv_theta[ncont], then cheb[deg][ncont][2]
    void* vec = nullptr;             // b, x, r, rr, dd, tt, cx, diag (levels >= 1, the cycle's precision)
    TxItem* d_tx = nullptr;          // transfers of the prefix to the next level
    long long tx_blocks[4] = {0, 0, 0, 0};
    ConsItem* d_cons = nullptr;      // constrained rows of all instances of the level
    int ncons = 0;
    long long cons_blocks = 0;
    CoarseItem* d_coarse = nullptr;  // direct coarsest solves of the instances after the prefix
    double* d_part = nullptr;        // their column-chunk partial sums
    int ncoarse = 0;
    long long coarse_blocks[2] = {0, 0};
  };
  std::vector<Level> lv;
  bool f32 = true;
  int deg = 0;
  int vm64 = 0, vm32 = 0;
};

void bmg_free(BatchMG* M) {
  if (!M) return;
  for (auto& L : M->lv) {
    if (L.bat) mns_batch_destroy(L.bat);
    for (void* p : {(void*)L.d_seg, (void*)L.d_coef, L.vec, (void*)L.d_tx, (void*)L.d_cons, (void*)L.d_coarse,
                    (void*)L.d_part})
      if (p) (void)hipFree(p);
  }
  delete M;
}

void bmg_counts(const BatchMG* M, int* v64, int* v32) {
  *v64 = M ? M->vm64 : 0;
  *v32 = M ? M->vm32 : 0;
}

template <typename T>
static hipError_t upload(T** dst, const std::vector<T>& src) {
  *dst = nullptr;
  if (src.empty()) return hipSuccess;
  hipError_t e = hipMalloc((void**)dst, src.size() * sizeof(T));
  if (e == hipSuccess) e = hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice);
  return e;
}

int bmg_setup(mns_batch* B, mns_handle* const* level0, const mns_solve_opts* o, bool f32, hipStream_t s,
              BatchMG** out) {
  *out = nullptr;
  const int count = (int)B->hs.size();
  std::vector<MG*> mg(count);
  size_t depth = 0;
  for (int i = 0; i < count; ++i) {
    mg[i] = (MG*)B->hs[i]->mg;
    if (!mg[i] || mg[i]->L.size() < 2 || !mg[i]->coarse_ready || mg[i]->L[0].h != level0[i])
      return MNS_ERR_UNSUPPORTED;
    depth = std::max(depth, mg[i]->L.size());
  }
  // members of every level: level 0 in the batch's order, the others the
  // deepest hierarchies first (stable), so that each level's members with a
  // coarser level are a prefix and are the next level's members, in order
  std::vector<int> order(count);
  for (int i = 0; i < count; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return mg[a]->L.size() > mg[b]->L.size(); });
  std::vector<std::vector<int>> mem(depth);
  for (int i = 0; i < count; ++i) mem[0].push_back(i);
  for (size_t l = 1; l < depth; ++l)
    for (int i : order)
      if (mg[i]->L.size() > l) mem[l].push_back(i);
  std::vector<std::vector<int>> pos(depth, std::vector<int>(count, -1));  // member index of instance i
  for (size_t l = 0; l < depth; ++l)
    for (size_t j = 0; j < mem[l].size(); ++j) pos[l][mem[l][j]] = (int)j;

  auto* M = new BatchMG();
  M->f32 = f32;
  M->deg = o->mg_smooth_degree;
  M->lv.resize(depth);
  const size_t rb = f32 ? sizeof(float) : sizeof(double);
  hipError_t e = hipSuccess;
  int rc = MNS_OK;
  auto fail = [&](const std::string& what) {
    B->err = "batched multigrid set-up: " + what + (e != hipSuccess ? std::string(": ") + hipGetErrorString(e) : "");
    bmg_free(M);
    return rc ? rc : MNS_ERR_HIP;
  };
  for (size_t l = 0; l < depth; ++l) {
    BatchMG::Level& Lv = M->lv[l];
    const std::vector<int>& ms = mem[l];
    Lv.count = (int)ms.size();
    Lv.off.assign(Lv.count + 1, 0);
    for (int j = 0; j < Lv.count; ++j) {
      const int i = ms[j];
      Lv.off[j + 1] = Lv.off[j] + mg[i]->L[l].n;
      if (mg[i]->L.size() > l + 1) Lv.ncont = j + 1;
    }
    Lv.n = Lv.off[Lv.count];
    Lv.ncn = Lv.off[Lv.ncont];
    if (l == 0)
      for (int j = 0; j < count; ++j)
        if (Lv.off[j] != B->offsets[j]) return fail("level-0 sizes differ from the batch's");
    // transfers of the prefix to level l + 1
    if (Lv.ncont > 0) {
      std::vector<TxItem> tx(Lv.ncont);
      long long acc[4] = {0, 0, 0, 0};
      for (int j = 0; j < Lv.ncont; ++j) {
        const int i = ms[j];
        TxItem& t = tx[j];
        t.X = mg[i]->T[l];
        restrict_passes(t.X, t.P, t.n);
        t.nnf = mg[i]->L[l].h->nnodes;
        t.tmp = mg[i]->L[l].tr;
        t.foff = Lv.off[j];
        t.coff = -1;  // set below from the next level's offsets
        const long long nb[4] = {(t.n[0] + 255) / 256, (t.n[1] + 255) / 256, (t.n[2] + 255) / 256,
                                 (t.nnf + 255) / 256};
        for (int p = 0; p < 4; ++p) {
          t.blk[p] = acc[p];
          acc[p] += nb[p];
        }
      }
      for (int p = 0; p < 4; ++p) Lv.tx_blocks[p] = acc[p];
      // the instances' first entries on level l + 1
      std::vector<long long> off1(mem[l + 1].size() + 1, 0);
      for (size_t j = 0; j < mem[l + 1].size(); ++j) off1[j + 1] = off1[j] + mg[mem[l + 1][j]]->L[l + 1].n;
      for (int j = 0; j < Lv.ncont; ++j) {
        if (pos[l + 1][ms[j]] < 0) return fail("level membership");
        tx[j].coff = off1[pos[l + 1][ms[j]]];
      }
      if ((e = upload(&Lv.d_tx, tx)) != hipSuccess) return fail("transfer items");
    }
    // constrained rows of every member
    {
      std::vector<ConsItem> ci;
      long long acc = 0;
      for (int j = 0; j < Lv.count; ++j) {
        const mns_handle* hl = mg[ms[j]]->L[l].h;
        if (hl->n_cons == 0) continue;
        ci.push_back(ConsItem{hl->d_cons, (long long)hl->n_cons, Lv.off[j], acc});
        acc += (hl->n_cons + 255) / 256;
      }
      Lv.ncons = (int)ci.size();
      Lv.cons_blocks = acc;
      if ((e = upload(&Lv.d_cons, ci)) != hipSuccess) return fail("constraint items");
    }
    if (l == 0) continue;  // level 0: smoothing and vectors belong to the batched solver
    // direct coarsest solves of the members after the prefix
    {
      std::vector<CoarseItem> co;
      std::vector<long long> poff;  // each item's first partial sum
      long long acc[2] = {0, 0}, nparts = 0;
      for (int j = Lv.ncont; j < Lv.count; ++j) {
        CoarseItem it{};
        if ((rc = coarse_item(mg[ms[j]]->coarse, &it)) || it.n != Lv.off[j + 1] - Lv.off[j])
          return fail("coarsest-level solve of instance " + std::to_string(ms[j]));
        it.off = Lv.off[j];
        poff.push_back(nparts);
        nparts += (long long)coarse_parts(it.n) * it.n;
        long long pb, sb;
        coarse_blocks(it.n, &pb, &sb);
        it.blk0 = acc[0];
        it.blk1 = acc[1];
        acc[0] += pb;
        acc[1] += sb;
        co.push_back(it);
      }
      Lv.ncoarse = (int)co.size();
      Lv.coarse_blocks[0] = acc[0];
      Lv.coarse_blocks[1] = acc[1];
      if (nparts > 0 && (e = hipMalloc((void**)&Lv.d_part, (size_t)nparts * sizeof(double))) != hipSuccess)
        return fail("coarse partial sums");
      for (size_t q = 0; q < co.size(); ++q) co[q].part = Lv.d_part + poff[q];
      if ((e = upload(&Lv.d_coarse, co)) != hipSuccess) return fail("coarse items");
    }
    if ((e = hipMalloc(&Lv.vec, 8 * (size_t)Lv.n * rb)) != hipSuccess) return fail("level vectors");
    if (Lv.ncont == 0) continue;
    // the prefix: its batch, segments, diagonals and Chebyshev scalars
    std::vector<mns_handle*> hs(Lv.ncont);
    std::vector<long long> seg(2 * (size_t)(Lv.ncont + 1), 0);
    std::vector<double> lam(Lv.ncont);
    char* diag = (char*)Lv.vec + 7 * (size_t)Lv.n * rb;
    for (int j = 0; j < Lv.ncont; ++j) {
      const MGLevel& ml = mg[ms[j]]->L[l];
      hs[j] = ml.h;
      lam[j] = ml.lmax;
      seg[j + 1] = seg[j] + (ml.n + kBChunk - 1) / kBChunk;
      seg[Lv.ncont + 1 + j] = Lv.off[j];
      const void* dsrc = f32 ? (const void*)ml.h->d_diag32 : (const void*)ml.h->d_diag64;
      if ((e = hipMemcpyAsync(diag + (size_t)Lv.off[j] * rb, dsrc, (size_t)ml.n * rb, hipMemcpyDeviceToDevice, s)) !=
          hipSuccess)
        return fail("diagonals");
    }
    seg[2 * (size_t)Lv.ncont + 1] = Lv.ncn;
    Lv.nblk = seg[Lv.ncont];
    if ((rc = mns_batch_create(hs.data(), Lv.ncont, &Lv.bat))) return fail("level batch: " + hs[0]->err);
    if ((e = upload(&Lv.d_seg, seg)) != hipSuccess) return fail("segments");
    double* d_lam = nullptr;
    if ((e = upload(&d_lam, lam)) != hipSuccess) return fail("spectra");
    if ((e = hipMalloc((void**)&Lv.d_coef, (size_t)Lv.ncont * (1 + 2 * (size_t)std::max(M->deg, 1)) *
                                               sizeof(double))) != hipSuccess) {
      (void)hipFree(d_lam);
      return fail("Chebyshev scalars");
    }
    hipLaunchKernelGGL(k_bmg_coef, dim3(1), dim3(256), 0, s, (const double*)d_lam, Lv.ncont, M->deg,
                       o->cheb_lambda_factor, o->mg_smooth_range, Lv.d_coef, Lv.d_coef + Lv.ncont);
    e = hipStreamSynchronize(s);
    (void)hipFree(d_lam);
    if (e != hipSuccess) return fail("Chebyshev scalars");
  }
  *out = M;
  return MNS_OK;
}

template <typename Real>
static int bmg_jac(BatchMG* M, BatchMG::Level& Lv, const Real* src, Real* dst, hipStream_t s) {
  ++(sizeof(Real) == 8 ? M->vm64 : M->vm32);
  return launch_batch_jacobian<Real>(Lv.bat, src, dst, s);
}

// x = Chebyshev polynomial of degree deg in D^-1 J applied to b (from zero),
// on the level's prefix
template <typename Real>
static int bmg_poly(BatchMG* M, BatchMG::Level& Lv, const Real* b, Real* x, Real* rr, Real* dd, Real* tt,
                    const Real* diag, hipStream_t s) {
  const BSeg S{Lv.d_seg, Lv.d_seg + Lv.ncont + 1, Lv.ncont};
  const unsigned nb = (unsigned)Lv.nblk;
  hipLaunchKernelGGL(k_bcheb_init<Real>, dim3(nb), dim3(kBT), 0, s, S, b, diag, (const double*)Lv.d_coef, rr, dd, x);
  for (int k = 0; k < M->deg; ++k) {
    int rc;
    if ((rc = bmg_jac<Real>(M, Lv, dd, tt, s))) return rc;
    hipLaunchKernelGGL(k_bcheb_step<Real>, dim3(nb), dim3(kBT), 0, s, S, rr, (const Real*)tt, diag,
                       (const double*)(Lv.d_coef + Lv.ncont + (size_t)k * Lv.ncont * 2), dd, x);
  }
  return MNS_OK;
}

template <typename Real>
static void bmg_constrain(const BatchMG::Level& Lv, Real* v, hipStream_t s) {
  if (Lv.ncons)
    hipLaunchKernelGGL(k_bmg_constraints<Real>, dim3((unsigned)Lv.cons_blocks), dim3(256), 0, s,
                       (const ConsItem*)Lv.d_cons, Lv.ncons, v);
}

template <typename Real>
static void bmg_restrict(const BatchMG::Level& Lv, const Real* fine, Real* coarse, hipStream_t s) {
  for (int p = 0; p < 3; ++p)
    hipLaunchKernelGGL(k_bmg_restrict<Real>, dim3((unsigned)Lv.tx_blocks[p]), dim3(256), 0, s,
                       (const TxItem*)Lv.d_tx, Lv.ncont, p, fine, coarse);
}

template <typename Real>
static void bmg_prolong(const BatchMG::Level& Lv, const Real* coarse, Real* fine, hipStream_t s) {
  hipLaunchKernelGGL(k_bmg_prolong<Real>, dim3((unsigned)Lv.tx_blocks[3]), dim3(256), 0, s, (const TxItem*)Lv.d_tx,
                     Lv.ncont, coarse, fine);
}

template <typename Real>
static void bmg_axpy(const Real* a, Real beta, const Real* c, Real* o, long long n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_mg_axpy<Real>, dim3(grid_for(n)), dim3(256), 0, s, a, beta, c, o, n);
}

// the cycle from level l (>= 1) down: b -> x on every member of the level
template <typename Real>
static int bmg_cycle(BatchMG* M, size_t l, hipStream_t s) {
  BatchMG::Level& Lv = M->lv[l];
  const long long n = Lv.n;
  Real* v = (Real*)Lv.vec;
  Real *b = v, *x = v + n, *r = v + 2 * n, *rr = v + 3 * n, *dd = v + 4 * n, *tt = v + 5 * n, *cx = v + 6 * n;
  const Real* diag = v + 7 * n;
  int rc;
  if (Lv.ncont > 0) {
    BatchMG::Level& Lc = M->lv[l + 1];
    Real* vc = (Real*)Lc.vec;
    if ((rc = bmg_poly<Real>(M, Lv, b, x, rr, dd, tt, diag, s))) return rc;
    // residual, restricted with constrained rows zero on both levels
    if ((rc = bmg_jac<Real>(M, Lv, x, tt, s))) return rc;
    bmg_axpy<Real>(b, Real(-1), tt, r, Lv.ncn, s);
    bmg_constrain<Real>(Lv, r, s);
    bmg_restrict<Real>(Lv, r, vc, s);
    bmg_constrain<Real>(Lc, vc, s);
    if ((rc = bmg_cycle<Real>(M, l + 1, s))) return rc;
    // x += P x_c (constrained rows of the correction zero)
    bmg_prolong<Real>(Lv, vc + Lc.n, r, s);
    bmg_constrain<Real>(Lv, r, s);
    bmg_axpy<Real>(x, Real(1), r, x, Lv.ncn, s);
    // post-smoothing: x += poly(b - J x)
    if ((rc = bmg_jac<Real>(M, Lv, x, tt, s))) return rc;
    bmg_axpy<Real>(b, Real(-1), tt, r, Lv.ncn, s);
    if ((rc = bmg_poly<Real>(M, Lv, r, cx, rr, dd, tt, diag, s))) return rc;
    bmg_axpy<Real>(x, Real(1), cx, x, Lv.ncn, s);
  }
  if (Lv.ncoarse > 0 && (rc = coarse_apply_batch<Real>(Lv.d_coarse, Lv.ncoarse, Lv.coarse_blocks[0],
                                                        Lv.coarse_blocks[1], b, x, s)))
    return rc;
  return hipGetLastError() == hipSuccess ? MNS_OK : MNS_ERR_HIP;
}

template <typename Real>
int bmg_correction(BatchMG* M, Real* r0, Real* x0, Real* t0, hipStream_t s) {
  if (!M || M->lv.size() < 2 || (sizeof(Real) == 4) != M->f32) return MNS_ERR_INVALID_ARG;
  BatchMG::Level &L0 = M->lv[0], &L1 = M->lv[1];
  Real* v1 = (Real*)L1.vec;
  bmg_constrain<Real>(L0, r0, s);
  bmg_restrict<Real>(L0, r0, v1, s);
  bmg_constrain<Real>(L1, v1, s);
  int rc = bmg_cycle<Real>(M, 1, s);
  if (rc) return rc;
  bmg_prolong<Real>(L0, v1 + L1.n, t0, s);
  bmg_constrain<Real>(L0, t0, s);
  bmg_axpy<Real>(x0, Real(1), t0, x0, L0.n, s);
  return hipGetLastError() == hipSuccess ? MNS_OK : MNS_ERR_HIP;
}
template int bmg_correction<float>(BatchMG*, float*, float*, float*, hipStream_t);
template int bmg_correction<double>(BatchMG*, double*, double*, double*, hipStream_t);

}  // namespace mns

int mns_solve_impl(mns_handle* h, const double* rhs, double* x, const mns_solve_opts* o, mns_solve_report* rep,
                   hipStream_t s) {
  const auto t0 = std::chrono::steady_clock::now();
  const int m = o->restart;
  int rc = ensure_workspace(h, m);
  if (rc) return rc;
  Solver S = make_solver(h, s, h->ws_restart);
  // the preconditioner graph lives for this call only
  struct GraphGuard {
    Solver& S;
    ~GraphGuard() {
      if (S.gexec) (void)hipStreamSynchronize(S.s);
      S.release_graph();
    }
  } graph_guard{S};
  const size_t n = (size_t)h->ndofs;

  double lmax = 0;
  if (o->precond == MNS_PRECOND_MG || o->precond == MNS_PRECOND_MG64) {
    MG* mg = nullptr;
    if ((rc = mg_build(h, o->mg_levels, &mg))) return rc;
    if ((rc = mg_setup(h, mg, o, s))) return rc;
    S.mg = mg;
    lmax = mg->L[0].lmax;
  } else if (o->precond != -1) {
    if ((rc = cached_diagonal(h, s))) return rc;
    if ((rc = S.estimate_lambda(o->eig_iters, &lmax))) return rc;
  }
  rep->lambda_max = lmax;

  // ||b||
  double bn;
  hipLaunchKernelGGL(k_multidot, dim3(kRedBlocks), dim3(kRedThreads), 0, s, rhs, (long long)n, 1, rhs, S.parts(), 0);
  if ((rc = S.reduce(1)) || (rc = S.sync_read(1, &bn))) return rc;
  bn = std::sqrt(bn);
  if (!(bn > 0)) {
    if ((rc = launch_fill<double>(x, 0.0, (int64_t)n, s))) return set_error(h, rc, "fill");
    (void)hipStreamSynchronize(s);
    rep->status = MNS_OK;
    rep->rel_residual = 0;
    return MNS_OK;
  }
  const double target = o->rtol * bn;
  S.G = gm_view(h->d_gm, h->gm_m);
  S.zbuf = S.r;  // free during a cycle: the residual is read into V_0 at its start
  const double lam = lmax * o->cheb_lambda_factor;
  int total = 0, restarts = 0;
  double rnorm = 0, misc[GM_MISC];
  bool converged = false;
  while (total < o->maxit) {
    if ((rc = S.true_residual(rhs, x, S.r, &rnorm))) return rc;
    if (rnorm <= target) {
      converged = true;
      break;
    }
    hipLaunchKernelGGL(k_gm_start, dim3(grid_for(n)), dim3(256), 0, s, S.G, (const double*)S.r, rnorm, target, S.V,
                       (long long)n);
    // iterations in chunks between readbacks of the device state; the chunk
    // follows the observed convergence rate so that few iterations run past
    // convergence (they leave the state unchanged)
    const int cycle = std::min(m, o->maxit - total);
    int launched = 0, its = 0;
    double res0 = rnorm, res = rnorm;
    bool done = false;
    while (launched < cycle && !done) {
      int chunk = 1;
      if (its > 0 && res < res0 && res > target) {
        const double rate = std::log(res / res0) / its;  // < 0
        const double left = std::log(target / res) / rate;
        chunk = (int)std::max(1.0, std::min(8.0, std::floor(0.5 * left)));
      }
      chunk = std::min(chunk, cycle - launched);
      if ((rc = S.iterations(o, lam, chunk))) return rc;
      launched += chunk;
      if ((rc = S.read_state(misc))) return rc;
      if (misc[GM_BROKEN] != 0.0) return set_error(h, MNS_ERR_HIP, "non-finite value in FGMRES");
      its = (int)misc[GM_ITS];
      res = misc[GM_RES];
      done = misc[GM_DONE] != 0.0;
    }
    const int jj = (int)misc[GM_J];
    if (its < 1 || jj < 1) return set_error(h, MNS_ERR_HIP, "FGMRES cycle made no progress");
    total += its;
    S.vm64 += its * S.it_vm64;
    S.vm32 += its * S.it_vm32;
    // y = H^-1 g on the device, x += Z y
    hipLaunchKernelGGL(k_gm_backsub, dim3(1), dim3(64), 0, s, S.G, jj);
    hipLaunchKernelGGL(k_update_x, dim3(grid_for(n)), dim3(256), 0, s, (const double*)S.Z, (long long)n, jj,
                       (const double*)S.G.y, x);
    if (hipGetLastError() != hipSuccess) return set_error(h, MNS_ERR_HIP, "FGMRES update");
    ++restarts;
  }
  if (!converged) {
    if ((rc = S.true_residual(rhs, x, S.r, &rnorm))) return rc;
    converged = rnorm <= target;
  }
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return set_error(h, MNS_ERR_HIP, std::string("sync: ") + hipGetErrorString(e));
  rep->iterations = total;
  rep->restarts = restarts;
  rep->rel_residual = rnorm / bn;
  rep->vmults_f64 = S.vm64;
  rep->vmults_f32 = S.vm32;
  rep->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  rep->status = converged ? MNS_OK : MNS_ERR_NOT_CONVERGED;
  if (!converged) return set_error(h, MNS_ERR_NOT_CONVERGED, "FGMRES reached maxit");
  return MNS_OK;
}

namespace mns {

void mg_free(mns_handle* h) {
  MG* mg = (MG*)h->mg;
  if (!mg) return;
  for (size_t l = 0; l < mg->L.size(); ++l) {
    MGLevel& Lv = mg->L[l];
    if (Lv.b) (void)hipFree(Lv.b);
    if (Lv.inj) (void)hipFree(Lv.inj);
    if (Lv.tr) (void)hipFree(Lv.tr);
    if (Lv.cmask) (void)hipFree(Lv.cmask);
    if (l > 0 && Lv.h) mns_destroy(Lv.h);
  }
  if (mg->fine) mns_destroy(mg->fine);
  coarse_free(mg->coarse);
  for (void* p : mg->tables)
    if (p) (void)hipFree(p);
  delete mg;
  h->mg = nullptr;
}

int mg_levels(mns_handle* h, int* levels, hipStream_t) {
  MG* mg = nullptr;
  int rc = mg_build(h, 0, &mg);
  if (rc) return rc;
  *levels = (int)mg->L.size();
  return MNS_OK;
}

int mg_restrict64(mns_handle* h, int level, const double* x, double* y, hipStream_t s) {
  MG* mg = nullptr;
  int rc = mg_build(h, 0, &mg);
  if (rc) return rc;
  if (level < 0 || level + 1 >= (int)mg->L.size()) return set_error(h, MNS_ERR_INVALID_ARG, "no such multigrid level");
  if ((rc = mg_restrict<double>(mg->T[level], mg->L[level].tr, x, y, s)))
    return set_error(h, MNS_ERR_HIP, "restriction");
  return MNS_OK;
}

int mg_prolongate64(mns_handle* h, int level, const double* x, double* y, hipStream_t s) {
  MG* mg = nullptr;
  int rc = mg_build(h, 0, &mg);
  if (rc) return rc;
  if (level < 0 || level + 1 >= (int)mg->L.size()) return set_error(h, MNS_ERR_INVALID_ARG, "no such multigrid level");
  mns_handle* hf = mg->L[level].h;
  hipLaunchKernelGGL(k_mg_prolong<double>, dim3((unsigned)((hf->nnodes + 255) / 256)), dim3(256), 0, s,
                     mg->T[level], x, y, (long long)hf->nnodes, 0, (const unsigned char*)nullptr);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? MNS_OK : set_error(h, MNS_ERR_HIP, std::string("prolongation: ") + hipGetErrorString(e));
}

}  // namespace mns
