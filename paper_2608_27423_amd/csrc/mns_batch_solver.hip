// Batched FGMRES: the instances of a batch solve J_i x_i = b_i together, in
// lockstep, every iteration one batched preconditioner application, one
// batched FP64 Jacobian application and batched Gram-Schmidt reductions over
// the concatenated vectors.  The arithmetic of each instance is that of
// mns_solve with the Jacobi-Chebyshev preconditioner (Sec. 3.4 smoother
// polynomial with the diagonal of Alg. Alg-diagonal); only the reduction
// order of the dot products differs.  Vector kernels work on blocks that never
// straddle two instances, so per-instance scalars are read once per block.
//
// The whole solver state lives on the device: per-instance Gram-Schmidt
// coefficients, Hessenberg columns, Givens rotations, residual estimates and
// convergence flags, plus the column j shared by the lockstep.  One iteration
// is therefore a fixed sequence of launches that reads j from the device; it
// is captured once per call into a HIP graph and replayed, and the host reads
// the state back once per chunk of iterations.  Instances that have converged
// are skipped by the Gram-Schmidt kernels and their next basis vectors are
// zero, so the preconditioner and the Jacobian map them to zero.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "mns_batch_vec.hpp"
#include "mns_internal.hpp"

namespace mns {
namespace {

constexpr int kBK = 32;            // register width of one column chunk of the dot kernels
constexpr int kBMaxRestart = 200;  // columns staged in LDS by the Gram-Schmidt kernels

// stride of the rows of partial and per-instance sums: K + 1 <= restart + 1
// values (one chunk up to restart 31)
inline int brow(int m) { return m + 2 > kBK + 1 ? m + 2 : kBK + 1; }

// ---------------------------------------------------------------------------
// Device state (doubles; count instances, restart m, Chebyshev degree deg):
// part[nblk][P] partial sums, hc[count][P] first projection (and w . w
// before it), h2[count][P] second projection (and w . w after the first),
// P = brow(m),
// n3[count] w . w after the optional third pass, cs/sn[count][m],
// g[count][m + 1], H[count][m + 1][m], y[count][m], sc[count] scale factors,
// cheb[deg][count][2], inv_theta[count], inst[count][BI_N], misc[BG_MISC].
// ---------------------------------------------------------------------------
enum {
  BG_J = 0,        // column of the next iteration (shared by the lockstep)
  BG_ALLDONE = 1,  // 1 once every instance met its target or broke down
  BG_BROKEN = 2,   // 1 after a non-finite norm (power iteration or Arnoldi)
  BG_WORST = 3,    // max over the unconverged instances of residual estimate / target
  BG_MISC = 8
};
enum {
  BI_DONE = 0,    // this cycle: residual estimate met the target (or w vanished)
  BI_TARGET = 1,  // rtol ||b_i||
  BI_BN = 2,      // ||b_i||
  BI_ITS = 3,     // iterations taken, all cycles
  BI_RES = 4,     // residual estimate |g_j| (true residual at a cycle start)
  BI_INVWN = 5,   // scale of the next basis vector (0 when done)
  BI_JN = 6,      // columns of this cycle
  BI_LAM = 7,     // power-iteration estimate of lambda_max
  BI_N = 8
};

struct BState {
  double *part, *hc, *h2, *n3, *cs, *sn, *g, *H, *y, *sc, *cheb, *inv_theta, *inst, *misc;
  int count, m, P;
};

size_t bstate_doubles(long long nblk, int count, int m, int deg) {
  const size_t c = (size_t)count, P = (size_t)brow(m);
  return (size_t)nblk * P + 2 * c * P + c + 2 * c * m + c * (m + 1) + c * (m + 1) * m + c * m + c +
         (size_t)deg * c * 2 + c + c * BI_N + BG_MISC;
}

BState bstate_view(double* base, long long nblk, int count, int m, int deg) {
  BState G;
  G.count = count;
  G.m = m;
  G.P = brow(m);
  const size_t c = (size_t)count, P = (size_t)G.P;
  G.part = base;
  G.hc = G.part + (size_t)nblk * P;
  G.h2 = G.hc + c * P;
  G.n3 = G.h2 + c * P;
  G.cs = G.n3 + c;
  G.sn = G.cs + c * m;
  G.g = G.sn + c * m;
  G.H = G.g + c * (m + 1);
  G.y = G.H + c * (m + 1) * m;
  G.sc = G.y + c * m;
  G.cheb = G.sc + c;
  G.inv_theta = G.cheb + (size_t)deg * c * 2;
  G.inst = G.inv_theta + c;
  G.misc = G.inst + c * BI_N;  // misc follows inst, so that one copy reads both
  return G;
}

__device__ inline double& inst_at(const BState& G, int i, int f) { return G.inst[(size_t)i * BI_N + f]; }
__device__ inline bool all_done(const BState& G) { return G.misc[BG_ALLDONE] != 0.0; }
__device__ inline int col_j(const BState& G) { return (int)G.misc[BG_J]; }

// per-block sums of cnt thread values into part[blockIdx.x * P + k0 + k]
template <int MAXK>
__device__ inline void bsum_store(double (&v)[MAXK], int cnt, double* part, int P, int k0 = 0) {
  __shared__ double red[kBT / 64][MAXK];
  const int lane = threadIdx.x % 64, wid = threadIdx.x / 64;
#pragma unroll
  for (int k = 0; k < MAXK; ++k) {
    if (k < cnt) {
      double x = v[k];
      for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
      if (lane == 0) red[wid][k] = x;
    }
  }
  __syncthreads();
  if ((int)threadIdx.x < cnt) {
    double t = 0;
    for (int w = 0; w < kBT / 64; ++w) t += red[w][threadIdx.x];
    part[(long long)blockIdx.x * P + k0 + threadIdx.x] = t;
  }
}

// sums over instance i's blocks of part[.][0 .. cnt) in a fixed order, stored
// by thread 0 into out[0 .. cnt); ends with a barrier, so that shared-memory
// results are visible to every thread of the block
__device__ inline void instance_sums(const BSeg& S, const double* part, int P, int i, int cnt, double* out) {
  __shared__ double red[kBT];
  const long long b0 = S.bstart[i], b1 = S.bstart[i + 1];
  for (int k = 0; k < cnt; ++k) {
    double t = 0;
    for (long long b = b0 + threadIdx.x; b < b1; b += kBT) t += part[b * P + k];
    red[threadIdx.x] = t;
    __syncthreads();
    for (int off = kBT / 2; off > 0; off >>= 1) {
      if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[k] = red[0];
    __syncthreads();
  }
}

// ---- set-up kernels --------------------------------------------------------

// partial sums of w . w
__global__ __launch_bounds__(kBT) void k_bnorm(BSeg S, const double* __restrict__ w, double* __restrict__ part, int P) {
  int i;
  long long lo, hi;
  bseg_range(S, blockIdx.x, i, lo, hi);
  double acc[1] = {0};
  for (long long r = lo + threadIdx.x; r < hi; r += kBT) acc[0] += w[r] * w[r];
  bsum_store<1>(acc, 1, part, P);
}

// ||b_i||, the target rtol ||b_i||, sc = 1 (0 for a zero right-hand side, so
// that x_i = 0), iteration counts cleared
__global__ __launch_bounds__(kBT) void k_bgm_init(BSeg S, BState G, double rtol) {
  const int i = blockIdx.x;
  __shared__ double s[1];
  instance_sums(S, G.part, G.P, i, 1, s);
  if (threadIdx.x == 0) {
    const double bn = sqrt(s[0]);
    inst_at(G, i, BI_BN) = bn;
    inst_at(G, i, BI_TARGET) = rtol * bn;
    inst_at(G, i, BI_ITS) = 0.0;
    inst_at(G, i, BI_LAM) = 1.0;
    G.sc[i] = bn > 0 ? 1.0 : 0.0;
    if (i == 0)
      for (int k = 0; k < BG_MISC; ++k) G.misc[k] = 0.0;
  }
}

// y = sc[i] x; x and y may be the same vector
__global__ __launch_bounds__(kBT) void k_bscale(BSeg S, const double* x, const double* __restrict__ sc, double* y) {
  int i;
  long long lo, hi;
  bseg_range(S, blockIdx.x, i, lo, hi);
  const double a = sc[i];
  for (long long r = lo + threadIdx.x; r < hi; r += kBT) y[r] = a * x[r];
}

// start of the power iteration: sc = 1 / sqrt(n_i)
__global__ void k_bpower_start(BSeg S, BState G) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < S.count; i += gridDim.x * blockDim.x)
    G.sc[i] = 1.0 / sqrt((double)(S.off[i + 1] - S.off[i]));
}

// y = D^-1 t (power iteration), partial ||y||^2
__global__ __launch_bounds__(kBT) void k_bpower(BSeg S, const double* __restrict__ t, const double* __restrict__ diag,
                                                double* __restrict__ y, double* __restrict__ part, int P) {
  int i;
  long long lo, hi;
  bseg_range(S, blockIdx.x, i, lo, hi);
  double acc[1] = {0};
  for (long long q = lo + threadIdx.x; q < hi; q += kBT) {
    const double v = t[q] / diag[q];
    y[q] = v;
    acc[0] += v * v;
  }
  bsum_store<1>(acc, 1, part, P);
}

// lambda_i = ||D^-1 J v_i|| and sc = 1 / lambda_i; a breakdown sets BG_BROKEN
__global__ __launch_bounds__(kBT) void k_bpower_norm(BSeg S, BState G) {
  const int i = blockIdx.x;
  __shared__ double s[1];
  instance_sums(S, G.part, G.P, i, 1, s);
  if (threadIdx.x == 0) {
    const double lam = sqrt(s[0]);
    const bool ok = lam > 0 && isfinite(lam);
    inst_at(G, i, BI_LAM) = lam;
    G.sc[i] = ok ? 1.0 / lam : 0.0;
    if (!ok) G.misc[BG_BROKEN] = 1.0;
  }
}

// Chebyshev scalars per instance from lambda_i (BI_LAM)
__global__ void k_bcheb_coef(BState G, int deg, double lambda_factor, double range) {
  const int count = G.count;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x)
    cheb_scalars(inst_at(G, i, BI_LAM), lambda_factor, range, deg, count, i, G.inv_theta, G.cheb);
}

// ---- one cycle -------------------------------------------------------------

// r = b - t, partial ||r||^2
__global__ __launch_bounds__(kBT) void k_bresid(BSeg S, const double* __restrict__ b, const double* __restrict__ t,
                                                double* __restrict__ r, double* __restrict__ part, int P) {
  int i;
  long long lo, hi;
  bseg_range(S, blockIdx.x, i, lo, hi);
  double acc[1] = {0};
  for (long long q = lo + threadIdx.x; q < hi; q += kBT) {
    const double v = b[q] - t[q];
    r[q] = v;
    acc[0] += v * v;
  }
  bsum_store<1>(acc, 1, part, P);
}

// per instance at a cycle start: true residual norm, convergence, g = (||r||, 0, ...)
__global__ __launch_bounds__(kBT) void k_bgm_cycle(BSeg S, BState G) {
  const int i = blockIdx.x;
  __shared__ double s[1];
  instance_sums(S, G.part, G.P, i, 1, s);
  const double rn = sqrt(s[0]);
  const bool done = rn <= inst_at(G, i, BI_TARGET);
  double* gi = G.g + (size_t)i * (G.m + 1);
  for (int k = threadIdx.x; k <= G.m; k += kBT) gi[k] = (k == 0 && !done) ? rn : 0.0;
  if (threadIdx.x == 0) {
    inst_at(G, i, BI_RES) = rn;
    inst_at(G, i, BI_DONE) = done ? 1.0 : 0.0;
    inst_at(G, i, BI_JN) = 0.0;
    inst_at(G, i, BI_INVWN) = done ? 0.0 : 1.0 / rn;
  }
}

// the lockstep's flags from the per-instance ones: j = 0 at a cycle start
// (start = 1), every instance done, the worst ratio of estimate to target
__global__ __launch_bounds__(kBT) void k_bgm_flags(BState G, int start) {
  __shared__ double worst[kBT];
  int active = 0;
  double wr = 0.0;
  for (int i = threadIdx.x; i < G.count; i += kBT)
    if (inst_at(G, i, BI_DONE) == 0.0) {
      active = 1;
      wr = fmax(wr, inst_at(G, i, BI_RES) / fmax(inst_at(G, i, BI_TARGET), 1e-300));
    }
  worst[threadIdx.x] = wr;
  const int any = __syncthreads_or(active);
  if (threadIdx.x == 0) {
    double w = 0.0;
    for (int t = 0; t < kBT; ++t) w = fmax(w, worst[t]);
    if (start) G.misc[BG_J] = 0.0;
    G.misc[BG_WORST] = w;
    G.misc[BG_ALLDONE] = (!any || G.misc[BG_BROKEN] != 0.0) ? 1.0 : 0.0;
  }
}

// next basis vector V_j = inst.invwn * w (j already advanced; zero for done
// instances, so that the following preconditioner and Jacobian give zero)
__global__ __launch_bounds__(kBT) void k_bgm_next(BSeg S, BState G, double* __restrict__ V, long long N,
                                                  const double* __restrict__ w) {
  if (all_done(G)) return;
  int i;
  long long lo, hi;
  bseg_range(S, blockIdx.x, i, lo, hi);
  const double a = inst_at(G, i, BI_INVWN);
  double* vj = V + (long long)col_j(G) * N;
  for (long long r = lo + threadIdx.x; r < hi; r += kBT) vj[r] = a != 0.0 ? a * w[r] : 0.0;
}

// preconditioner input: V_j (cast to its precision) into a fixed buffer
template <typename To>
__global__ __launch_bounds__(kBT) void k_bgm_in(BSeg S, BState G, const double* __restrict__ V, long long N,
                                                To* __restrict__ dst) {
  if (all_done(G)) return;
  int i;
  long long lo, hi;
  bseg_range(S, blockIdx.x, i, lo, hi);
  const double* vj = V + (long long)col_j(G) * N;
  for (long long r = lo + threadIdx.x; r < hi; r += kBT) dst[r] = (To)vj[r];
}

// preconditioner output -> Z_j and the fixed FP64 input zbuf of the Jacobian
template <typename From>
__global__ __launch_bounds__(kBT) void k_bgm_out(BSeg S, BState G, const From* __restrict__ src, long long N,
                                                 double* __restrict__ Z, double* __restrict__ zbuf) {
  if (all_done(G)) return;
  int i;
  long long lo, hi;
  bseg_range(S, blockIdx.x, i, lo, hi);
  double* zj = Z + (long long)col_j(G) * N;
  for (long long r = lo + threadIdx.x; r < hi; r += kBT) {
    const double z = (double)src[r];
    zj[r] = z;
    zbuf[r] = z;
  }
}

// partial dots of w with V_0 .. V_{K-1} and w . w (entry K), K = j + 1
__global__ __launch_bounds__(kBT) void k_bgm_dots(BSeg S, BState G, const double* __restrict__ V, long long N,
                                                  const double* __restrict__ w) {
  if (all_done(G)) return;
  int i;
  long long lo, hi;
  bseg_range(S, blockIdx.x, i, lo, hi);
  if (inst_at(G, i, BI_DONE) != 0.0) return;
  const int K = col_j(G) + 1;
  // columns in chunks of kBK (one chunk up to restart 31), w . w at index K
  for (int c0 = 0; c0 <= K; c0 += kBK) {
    double acc[kBK];
#pragma unroll
    for (int k = 0; k < kBK; ++k) acc[k] = 0;
    for (long long r = lo + threadIdx.x; r < hi; r += kBT) {
      const double wr = w[r];
#pragma unroll
      for (int k = 0; k < kBK; ++k) {
        const int kk = c0 + k;
        if (kk < K) acc[k] += V[(long long)kk * N + r] * wr;
        if (kk == K) acc[k] += wr * wr;
      }
    }
    bsum_store<kBK>(acc, K + 1 - c0 < kBK ? K + 1 - c0 : kBK, G.part, G.P, c0);
    __syncthreads();  // bsum_store's shared rows are reused by the next chunk
  }
}

// w -= sum_k hc[i][k] V_k, then partial dots of the new w with V_k and w . w
__global__ __launch_bounds__(kBT) void k_bgm_axpy_dots(BSeg S, BState G, const double* __restrict__ V, long long N,
                                                       double* __restrict__ w) {
  if (all_done(G)) return;
  int i;
  long long lo, hi;
  bseg_range(S, blockIdx.x, i, lo, hi);
  if (inst_at(G, i, BI_DONE) != 0.0) return;
  const int K = col_j(G) + 1;
  const double* hrow = G.hc + (size_t)i * G.P;
  if (K + 1 > kBK) {
    // long restarts: the update with the coefficients staged in LDS, then the
    // dots of the new w in chunks (each thread re-reads only its own rows)
    __shared__ double hs[kBMaxRestart + 1];
    for (int k = threadIdx.x; k < K; k += kBT) hs[k] = hrow[k];
    __syncthreads();
    for (long long r = lo + threadIdx.x; r < hi; r += kBT) {
      double x = w[r];
      for (int k = 0; k < K; ++k) x -= hs[k] * V[(long long)k * N + r];
      w[r] = x;
    }
    for (int c0 = 0; c0 <= K; c0 += kBK) {
      double acc[kBK];
#pragma unroll
      for (int k = 0; k < kBK; ++k) acc[k] = 0;
      for (long long r = lo + threadIdx.x; r < hi; r += kBT) {
        const double x = w[r];
#pragma unroll
        for (int k = 0; k < kBK; ++k) {
          const int kk = c0 + k;
          if (kk < K) acc[k] += V[(long long)kk * N + r] * x;
          if (kk == K) acc[k] += x * x;
        }
      }
      bsum_store<kBK>(acc, K + 1 - c0 < kBK ? K + 1 - c0 : kBK, G.part, G.P, c0);
      __syncthreads();
    }
    return;
  }
  double hh[kBK], acc[kBK];
#pragma unroll
  for (int k = 0; k < kBK; ++k) {
    hh[k] = 0;
    if (k < K) hh[k] = hrow[k];
    acc[k] = 0;
  }
  for (long long r = lo + threadIdx.x; r < hi; r += kBT) {
    double v[kBK];
    double x = w[r];
#pragma unroll
    for (int k = 0; k < kBK; ++k) {
      v[k] = 0;
      if (k < K) v[k] = V[(long long)k * N + r];
      x -= hh[k] * v[k];
    }
    w[r] = x;
#pragma unroll
    for (int k = 0; k < kBK; ++k) {
      if (k < K) acc[k] += v[k] * x;
      if (k == K) acc[k] += x * x;
    }
  }
  bsum_store<kBK>(acc, K + 1, G.part, G.P);
}

// reorthogonalization (DGKS) where the projected norm dropped below 0.7 of the
// norm before the projection: w -= sum_k h2[i][k] V_k, partial ||w||^2
__device__ inline bool reorth(const BState& G, int i, int K) {
  return sqrt(G.h2[(size_t)i * G.P + K]) < 0.7 * sqrt(G.hc[(size_t)i * G.P + K]);
}

__global__ __launch_bounds__(kBT) void k_bgm_reorth(BSeg S, BState G, const double* __restrict__ V, long long N,
                                                    double* __restrict__ w) {
  if (all_done(G)) return;
  int i;
  long long lo, hi;
  bseg_range(S, blockIdx.x, i, lo, hi);
  const int K = col_j(G) + 1;
  if (inst_at(G, i, BI_DONE) != 0.0 || !reorth(G, i, K)) return;
  const double* hrow = G.h2 + (size_t)i * G.P;
  double acc[1] = {0};
  if (K > kBK) {
    __shared__ double hs[kBMaxRestart + 1];
    for (int k = threadIdx.x; k < K; k += kBT) hs[k] = hrow[k];
    __syncthreads();
    for (long long r = lo + threadIdx.x; r < hi; r += kBT) {
      double x = w[r];
      for (int k = 0; k < K; ++k) x -= hs[k] * V[(long long)k * N + r];
      w[r] = x;
      acc[0] += x * x;
    }
    bsum_store<1>(acc, 1, G.part, G.P);
    return;
  }
  double hh[kBK];
#pragma unroll
  for (int k = 0; k < kBK; ++k) {
    hh[k] = 0;
    if (k < K) hh[k] = hrow[k];
  }
  for (long long r = lo + threadIdx.x; r < hi; r += kBT) {
    double x = w[r];
#pragma unroll
    for (int k = 0; k < kBK; ++k)
      if (k < K) x -= hh[k] * V[(long long)k * N + r];
    w[r] = x;
    acc[0] += x * x;
  }
  bsum_store<1>(acc, 1, G.part, G.P);
}

// per-instance sums of the partial sums (block i = instance i): which 0:
// hc[i][0 .. K], 1: h2[i][0 .. K], 2: n3[i] (only where the third pass ran)
__global__ __launch_bounds__(kBT) void k_bgm_reduce(BSeg S, BState G, int which) {
  if (all_done(G)) return;
  const int i = blockIdx.x;
  if (inst_at(G, i, BI_DONE) != 0.0) return;
  const int K = col_j(G) + 1;
  if (which == 2 && !reorth(G, i, K)) return;
  double* out = which == 0 ? G.hc + (size_t)i * G.P : which == 1 ? G.h2 + (size_t)i * G.P : G.n3 + i;
  instance_sums(S, G.part, G.P, i, which == 2 ? 1 : K + 1, out);
}

// Hessenberg column, Givens rotations and residual estimate of column j for
// every unconverged instance (one thread each; products not contracted, as
// in the single-instance solver), then the lockstep advances j
__global__ __launch_bounds__(kBT) void k_bgm_givens(BState G) {
#pragma clang fp contract(off)
  if (all_done(G)) return;
  const int j = col_j(G), K = j + 1, m = G.m;
  int broken = 0;
  for (int i = threadIdx.x; i < G.count; i += kBT) {
    if (inst_at(G, i, BI_DONE) != 0.0) continue;
    double* hcol = G.hc + (size_t)i * G.P;
    const double* h2 = G.h2 + (size_t)i * G.P;
    double wn;
    if (reorth(G, i, K)) {
      wn = sqrt(G.n3[i]);
      for (int k = 0; k < K; ++k) hcol[k] += h2[k];
    } else {
      wn = sqrt(h2[K]);
    }
    hcol[K] = wn;
    if (!isfinite(wn)) {
      broken = 1;
      inst_at(G, i, BI_DONE) = 1.0;
      inst_at(G, i, BI_INVWN) = 0.0;
      continue;
    }
    double* cs = G.cs + (size_t)i * m;
    double* sn = G.sn + (size_t)i * m;
    double* g = G.g + (size_t)i * (m + 1);
    for (int k = 0; k < j; ++k) {
      const double a = cs[k] * hcol[k] + sn[k] * hcol[k + 1];
      const double b = -sn[k] * hcol[k] + cs[k] * hcol[k + 1];
      hcol[k] = a;
      hcol[k + 1] = b;
    }
    const double den = hypot(hcol[j], hcol[j + 1]);
    cs[j] = den > 0 ? hcol[j] / den : 1.0;
    sn[j] = den > 0 ? hcol[j + 1] / den : 0.0;
    hcol[j] = den;
    hcol[j + 1] = 0.0;
    g[j + 1] = -sn[j] * g[j];
    g[j] = cs[j] * g[j];
    double* H = G.H + (size_t)i * (m + 1) * m;
    for (int k = 0; k <= j; ++k) H[(size_t)k * m + j] = hcol[k];
    const double res = fabs(g[j + 1]);
    const bool done = res <= inst_at(G, i, BI_TARGET) || wn == 0;
    inst_at(G, i, BI_JN) = (double)(j + 1);
    inst_at(G, i, BI_ITS) += 1.0;
    inst_at(G, i, BI_RES) = res;
    inst_at(G, i, BI_DONE) = done ? 1.0 : 0.0;
    inst_at(G, i, BI_INVWN) = done ? 0.0 : 1.0 / wn;
  }
  __shared__ double worst[kBT];
  int active = 0;
  double wr = 0.0;
  for (int i = threadIdx.x; i < G.count; i += kBT)
    if (inst_at(G, i, BI_DONE) == 0.0) {
      active = 1;
      wr = fmax(wr, inst_at(G, i, BI_RES) / fmax(inst_at(G, i, BI_TARGET), 1e-300));
    }
  worst[threadIdx.x] = wr;
  const int any = __syncthreads_or(active);
  const int brk = __syncthreads_or(broken);
  if (threadIdx.x == 0) {
    double w = 0.0;
    for (int t = 0; t < kBT; ++t) w = fmax(w, worst[t]);
    G.misc[BG_WORST] = w;
    G.misc[BG_J] = (double)(j + 1);
    if (brk) G.misc[BG_BROKEN] = 1.0;
    if (!any || brk) G.misc[BG_ALLDONE] = 1.0;
  }
}

// y_i = H_i^-1 g_i (upper triangular, JN_i columns), one thread per instance
__global__ void k_bgm_backsub(BState G) {
#pragma clang fp contract(off)
  const int m = G.m;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < G.count; i += gridDim.x * blockDim.x) {
    const int jn = (int)inst_at(G, i, BI_JN);
    const double* H = G.H + (size_t)i * (m + 1) * m;
    const double* g = G.g + (size_t)i * (m + 1);
    double* y = G.y + (size_t)i * m;
    for (int a = jn - 1; a >= 0; --a) {
      double sum = g[a];
      for (int k = a + 1; k < jn; ++k) sum -= H[(size_t)a * m + k] * y[k];
      const double d = H[(size_t)a * m + a];
      y[a] = d != 0 ? sum / d : 0.0;
    }
  }
}

// x_i += sum_{k < JN_i} y_i[k] Z_k
__global__ __launch_bounds__(kBT) void k_bgm_update(BSeg S, BState G, const double* __restrict__ Z, long long N,
                                                    double* __restrict__ x) {
  int i;
  long long lo, hi;
  bseg_range(S, blockIdx.x, i, lo, hi);
  const int jn = (int)inst_at(G, i, BI_JN);
  const double* y = G.y + (size_t)i * G.m;
  for (long long r = lo + threadIdx.x; r < hi; r += kBT) {
    double a = x[r];
    for (int k = 0; k < jn; ++k) a += y[k] * Z[(long long)k * N + r];
    x[r] = a;
  }
}

// final true residual norm per instance into inst.res
__global__ __launch_bounds__(kBT) void k_bgm_final(BSeg S, BState G) {
  const int i = blockIdx.x;
  __shared__ double s[1];
  instance_sums(S, G.part, G.P, i, 1, s);
  if (threadIdx.x == 0) inst_at(G, i, BI_RES) = sqrt(s[0]);
}

struct BatchSolver {
  mns_batch* B;
  hipStream_t s;
  int count, m;
  long long N, nblk;
  unsigned nb;
  BSeg S;
  BState G;
  const mns_solve_opts* o;
  double *V, *Z, *w, *r, *t, *diag64, *cb, *cr, *cd, *cx, *ct, *mr64, *mx64;
  float *b32, *x32, *r32, *d32, *t32, *diag32, *mr32, *mx32;
  mns_batch* F = nullptr;  // multigrid: the batch of the level-0 operators
  BatchMG* bmg = nullptr;  // multigrid: the batched coarse levels (null: corrections per instance)
  int vm64 = 0, vm32 = 0;
  int it_vm64 = 0, it_vm32 = 0;  // Jacobian applications of one iteration
  hipGraphExec_t gexec = nullptr;

  int fail(int code, const std::string& msg) {
    B->err = msg;
    return code;
  }
  int check(const char* what) {
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? MNS_OK : fail(MNS_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
  }
  int jac64(const double* src, double* dst, hipStream_t st) {
    ++vm64;
    return launch_batch_jacobian<double>(B, src, dst, st);
  }
  int jac32(const float* src, float* dst, hipStream_t st) {
    ++vm32;
    return launch_batch_jacobian<float>(B, src, dst, st);
  }
  template <typename Real>
  int jac_fine(const Real* src, Real* dst, hipStream_t st) {
    ++(sizeof(Real) == 8 ? vm64 : vm32);
    const int rc = launch_batch_jacobian<Real>(F, src, dst, st);
    return rc ? fail(rc, F->err) : MNS_OK;
  }

  // x = Chebyshev polynomial of degree mg_smooth_degree in D0^-1 J0 applied
  // to b (from zero), J0, D0 the level-0 operators and diagonals
  template <typename Real>
  int mg_poly(const Real* b, Real* x, Real* rr, Real* dd, Real* tt, const Real* diag, hipStream_t st) {
    hipLaunchKernelGGL(k_bcheb_init<Real>, dim3(nb), dim3(kBT), 0, st, S, b, diag, (const double*)G.inv_theta, rr, dd,
                       x);
    for (int k = 0; k < o->mg_smooth_degree; ++k) {
      int rc;
      if ((rc = jac_fine<Real>(dd, tt, st))) return rc;
      hipLaunchKernelGGL(k_bcheb_step<Real>, dim3(nb), dim3(kBT), 0, st, S, rr, (const Real*)tt, diag,
                         (const double*)(G.cheb + (size_t)k * count * 2), dd, x);
    }
    return check("batch multigrid smoothing");
  }

  // one V-cycle (the single-instance cycle's steps): pre-smoothing on the
  // finest level of every instance, batched; residual; per instance the
  // coarse-grid correction (restriction, the cycle from level 1 with its
  // FP64 coarsest level, prolongation); post-smoothing, batched
  template <typename Real>
  int mg_vcycle(const Real* b, Real* x, Real* res, Real* xc, Real* rr, Real* dd, Real* tt, const Real* diag,
                hipStream_t st) {
    int rc;
    if ((rc = mg_poly<Real>(b, x, rr, dd, tt, diag, st))) return rc;
    if ((rc = jac_fine<Real>(x, tt, st))) return rc;
    hipLaunchKernelGGL(k_baxpy<Real>, dim3(nb), dim3(kBT), 0, st, S, b, Real(-1), (const Real*)tt, res);
    if ((rc = check("batch multigrid residual"))) return rc;
    if (bmg) {
      if ((rc = bmg_correction<Real>(bmg, res, x, tt, st))) return fail(rc, "batched coarse-grid correction");
    } else {
      for (int i = 0; i < count; ++i) {
        const long long off = B->offsets[i];
        mns_handle* h0 = B->mg_fine_hs[i];
        if ((rc = launch_constraints<Real>(h0, res + off, res + off, Real(0), 1, st)))
          return fail(rc, "batch multigrid constraints");
        if ((rc = mg_instance_correction<Real>(B->hs[i], res + off, x + off, o, st)))
          return fail(rc, "batch multigrid, instance " + std::to_string(i) + ": " + B->hs[i]->err);
      }
    }
    if ((rc = jac_fine<Real>(x, tt, st))) return rc;
    hipLaunchKernelGGL(k_baxpy<Real>, dim3(nb), dim3(kBT), 0, st, S, b, Real(-1), (const Real*)tt, res);
    if ((rc = mg_poly<Real>(res, xc, rr, dd, tt, diag, st))) return rc;
    hipLaunchKernelGGL(k_baxpy<Real>, dim3(nb), dim3(kBT), 0, st, S, (const Real*)x, Real(1), (const Real*)xc, x);
    return check("batch multigrid update");
  }
  // inst and misc -> host (one synchronization)
  int read_state() {
    const size_t cnt = (size_t)count * BI_N + BG_MISC;
    hipError_t e = hipMemcpyAsync(B->h_small, G.inst, cnt * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e == hipSuccess ? MNS_OK : fail(MNS_ERR_HIP, std::string("batch readback: ") + hipGetErrorString(e));
  }
  double inst(int i, int f) const { return B->h_small[(size_t)i * BI_N + f]; }
  double misc(int f) const { return B->h_small[(size_t)count * BI_N + f]; }

  // the preconditioner between its fixed buffers (precond -1: copy)
  int precondition(hipStream_t st) {
    const int deg = o->cheb_degree;
    int rc;
    if (o->precond == MNS_PRECOND_MG64) {
      hipLaunchKernelGGL(k_bgm_in<double>, dim3(nb), dim3(kBT), 0, st, S, G, (const double*)V, N, cb);
      return mg_vcycle<double>(cb, cx, mr64, mx64, cr, cd, ct, diag64, st);
    }
    if (o->precond == MNS_PRECOND_MG) {
      hipLaunchKernelGGL(k_bgm_in<float>, dim3(nb), dim3(kBT), 0, st, S, G, (const double*)V, N, b32);
      return mg_vcycle<float>(b32, x32, mr32, mx32, r32, d32, t32, diag32, st);
    }
    if (o->precond == -1) {
      hipLaunchKernelGGL(k_bgm_in<double>, dim3(nb), dim3(kBT), 0, st, S, G, (const double*)V, N, cx);
      return check("batch copy");
    }
    if (o->precond == MNS_F64) {
      hipLaunchKernelGGL(k_bgm_in<double>, dim3(nb), dim3(kBT), 0, st, S, G, (const double*)V, N, cb);
      hipLaunchKernelGGL(k_bcheb_init<double>, dim3(nb), dim3(kBT), 0, st, S, (const double*)cb,
                         (const double*)diag64, (const double*)G.inv_theta, cr, cd, cx);
      for (int k = 0; k < deg; ++k) {
        if ((rc = jac64(cd, ct, st))) return rc;
        hipLaunchKernelGGL(k_bcheb_step<double>, dim3(nb), dim3(kBT), 0, st, S, cr, (const double*)ct,
                           (const double*)diag64, (const double*)(G.cheb + (size_t)k * count * 2), cd, cx);
      }
      return check("batch Chebyshev");
    }
    hipLaunchKernelGGL(k_bgm_in<float>, dim3(nb), dim3(kBT), 0, st, S, G, (const double*)V, N, b32);
    hipLaunchKernelGGL(k_bcheb_init<float>, dim3(nb), dim3(kBT), 0, st, S, (const float*)b32, (const float*)diag32,
                       (const double*)G.inv_theta, r32, d32, x32);
    for (int k = 0; k < deg; ++k) {
      if ((rc = jac32(d32, t32, st))) return rc;
      hipLaunchKernelGGL(k_bcheb_step<float>, dim3(nb), dim3(kBT), 0, st, S, r32, (const float*)t32,
                         (const float*)diag32, (const double*)(G.cheb + (size_t)k * count * 2), d32, x32);
    }
    return check("batch Chebyshev");
  }

  // One lockstep iteration as a fixed sequence of launches (j is read from
  // the device): preconditioner, FP64 Jacobian, Gram-Schmidt with the
  // optional reorthogonalization, Givens, next basis vector.
  int mg_counts(int* a64, int* a32) {
    bmg_counts(bmg, a64, a32);
    for (int i = 0; i < count; ++i) {
      int c64, c32;
      mg_instance_counts(B->hs[i], &c64, &c32);
      *a64 += c64;
      *a32 += c32;
    }
    return MNS_OK;
  }

  int iteration(hipStream_t st) {
    const int v64 = vm64, v32 = vm32;
    int m64 = 0, m32 = 0;
    const bool mgp = o->precond == MNS_PRECOND_MG || o->precond == MNS_PRECOND_MG64;
    if (mgp) mg_counts(&m64, &m32);
    int rc = precondition(st);
    if (rc) return rc;
    if (mgp) {
      // Jacobian applications of the instances' own cycles (coarse levels)
      int a64, a32;
      mg_counts(&a64, &a32);
      vm64 += a64 - m64;
      vm32 += a32 - m32;
    }
    double* zbuf = r;  // free during a cycle: the residual is read into V_0 at its start
    if (o->precond == MNS_F32 || o->precond == MNS_PRECOND_MG)
      hipLaunchKernelGGL(k_bgm_out<float>, dim3(nb), dim3(kBT), 0, st, S, G, (const float*)x32, N, Z, zbuf);
    else
      hipLaunchKernelGGL(k_bgm_out<double>, dim3(nb), dim3(kBT), 0, st, S, G, (const double*)cx, N, Z, zbuf);
    if ((rc = jac64(zbuf, w, st))) return rc;
    hipLaunchKernelGGL(k_bgm_dots, dim3(nb), dim3(kBT), 0, st, S, G, (const double*)V, N, (const double*)w);
    hipLaunchKernelGGL(k_bgm_reduce, dim3(count), dim3(kBT), 0, st, S, G, 0);
    hipLaunchKernelGGL(k_bgm_axpy_dots, dim3(nb), dim3(kBT), 0, st, S, G, (const double*)V, N, w);
    hipLaunchKernelGGL(k_bgm_reduce, dim3(count), dim3(kBT), 0, st, S, G, 1);
    hipLaunchKernelGGL(k_bgm_reorth, dim3(nb), dim3(kBT), 0, st, S, G, (const double*)V, N, w);
    hipLaunchKernelGGL(k_bgm_reduce, dim3(count), dim3(kBT), 0, st, S, G, 2);
    hipLaunchKernelGGL(k_bgm_givens, dim3(1), dim3(kBT), 0, st, G);
    hipLaunchKernelGGL(k_bgm_next, dim3(nb), dim3(kBT), 0, st, S, G, V, N, (const double*)w);
    if ((rc = check("batch FGMRES iteration"))) return rc;
    it_vm64 = vm64 - v64;
    it_vm32 = vm32 - v32;
    vm64 = v64;  // counted by the caller per iteration that did work
    vm32 = v32;
    return MNS_OK;
  }

  int capture() {
    if (!B->cap && hipStreamCreateWithFlags(&B->cap, hipStreamNonBlocking) != hipSuccess)
      return fail(MNS_ERR_HIP, "batch capture stream");
    hipError_t e = hipStreamBeginCapture(B->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return fail(MNS_ERR_HIP, std::string("begin capture: ") + hipGetErrorString(e));
    const int rc = iteration(B->cap);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(B->cap, &graph);
    if (rc) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc;
    }
    if (e != hipSuccess) return fail(MNS_ERR_HIP, std::string("end capture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
      gexec = nullptr;
      return fail(MNS_ERR_HIP, std::string("graph instantiate: ") + hipGetErrorString(e));
    }
    return MNS_OK;
  }

  int iterations(int n) {
    int rc;
    if (o->use_graph) {
      if (!gexec && (rc = capture())) return rc;
      for (int k = 0; k < n; ++k) {
        const hipError_t e = hipGraphLaunch(gexec, s);
        if (e != hipSuccess) return fail(MNS_ERR_HIP, std::string("graph launch: ") + hipGetErrorString(e));
      }
      return MNS_OK;
    }
    for (int k = 0; k < n; ++k)
      if ((rc = iteration(s))) return rc;
    return MNS_OK;
  }

  ~BatchSolver() {
    if (gexec) {
      (void)hipStreamSynchronize(s);
      (void)hipGraphExecDestroy(gexec);
    }
  }
};

}  // namespace

void batch_solver_free(mns_batch* b) {
  if (b->d_seg) (void)hipFree(b->d_seg);
  if (b->ws) (void)hipFree(b->ws);
  if (b->ws32) (void)hipFree(b->ws32);
  if (b->d_small) (void)hipFree(b->d_small);
  if (b->h_small) (void)hipHostFree(b->h_small);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  b->d_seg = nullptr;
  b->ws = nullptr;
  b->ws32 = nullptr;
  b->d_small = nullptr;
  b->h_small = nullptr;
  b->cap = nullptr;
  b->ws_m = 0;
  b->small_doubles = 0;
}

int batch_solve_impl(mns_batch* B, const double* rhs, double* x, const mns_solve_opts* o, mns_solve_report* reps,
                     hipStream_t s) {
  const auto t0 = std::chrono::steady_clock::now();
  const int count = (int)B->hs.size();
  const long long N = B->ndofs;
  const bool mgp = o->precond == MNS_PRECOND_MG || o->precond == MNS_PRECOND_MG64;
  const int m = o->restart, deg = std::max(o->cheb_degree, mgp ? o->mg_smooth_degree : 1);
  hipError_t e;
  if (m < 1 || m > kBMaxRestart) return MNS_ERR_INVALID_ARG;
  // segmentation of the concatenated vectors into blocks of one instance
  if (!B->d_seg) {
    std::vector<long long> seg(2 * (size_t)(count + 1), 0);
    for (int i = 0; i < count; ++i) {
      const long long n = B->hs[i]->ndofs;
      seg[i + 1] = seg[i] + (n + kBChunk - 1) / kBChunk;
      seg[count + 1 + i] = B->offsets[i];
    }
    seg[2 * count + 1] = N;
    B->nvblk = seg[count];
    if ((e = hipMalloc((void**)&B->d_seg, seg.size() * sizeof(long long))) != hipSuccess ||
        (e = hipMemcpy(B->d_seg, seg.data(), seg.size() * sizeof(long long), hipMemcpyHostToDevice)) != hipSuccess) {
      B->err = std::string("batch segments: ") + hipGetErrorString(e);
      return MNS_ERR_HIP;
    }
  }
  // solver state: sized for the largest restart and degree seen so far
  const size_t need = bstate_doubles(B->nvblk, count, m, deg);
  if (B->small_doubles < need) {
    if (B->d_small) (void)hipFree(B->d_small);
    if (B->h_small) (void)hipHostFree(B->h_small);
    B->d_small = nullptr;
    B->h_small = nullptr;
    B->small_doubles = 0;
    if ((e = hipMalloc((void**)&B->d_small, need * sizeof(double))) != hipSuccess ||
        (e = hipHostMalloc((void**)&B->h_small, ((size_t)count * BI_N + BG_MISC) * sizeof(double),
                           hipHostMallocDefault)) != hipSuccess) {
      B->err = std::string("batch solver state: ") + hipGetErrorString(e);
      return MNS_ERR_HIP;
    }
    B->small_doubles = need;
  }
  if (B->ws_m < m) {
    if (B->ws) (void)hipFree(B->ws);
    if (B->ws32) (void)hipFree(B->ws32);
    B->ws = nullptr;
    B->ws32 = nullptr;
    B->ws_m = 0;
    if ((e = hipMalloc((void**)&B->ws, (size_t)(2 * m + 12) * N * sizeof(double))) != hipSuccess ||
        (e = hipMalloc((void**)&B->ws32, 8 * (size_t)N * sizeof(float))) != hipSuccess) {
      B->err = std::string("hipMalloc batch workspace: ") + hipGetErrorString(e);
      return MNS_ERR_HIP;
    }
    B->ws_m = m;
  }
  BatchSolver W;
  W.B = B;
  W.s = s;
  W.o = o;
  W.count = count;
  W.m = m;
  W.N = N;
  W.nblk = B->nvblk;
  W.nb = (unsigned)B->nvblk;
  W.S = BSeg{B->d_seg, B->d_seg + count + 1, count};
  W.G = bstate_view(B->d_small, B->nvblk, count, m, deg);
  W.V = B->ws;
  W.Z = W.V + (size_t)(m + 1) * N;
  W.w = W.Z + (size_t)m * N;
  W.r = W.w + N;
  W.t = W.r + N;
  W.diag64 = W.t + N;
  W.cb = W.diag64 + N;
  W.cx = W.cb + N;
  W.cr = W.cx + N;
  W.cd = W.cr + N;
  W.ct = W.cd + N;
  W.mr64 = W.ct + N;
  W.mx64 = W.mr64 + N;
  W.b32 = B->ws32;
  W.x32 = W.b32 + N;
  W.r32 = W.x32 + N;
  W.d32 = W.r32 + N;
  W.t32 = W.d32 + N;
  W.diag32 = W.t32 + N;
  W.mr32 = W.diag32 + N;
  W.mx32 = W.mr32 + N;
  const unsigned nb = W.nb;
  const BSeg& S = W.S;
  const BState& G = W.G;
  int rc;

  // ||b_i||, targets, x_i = 0 where b_i = 0
  hipLaunchKernelGGL(k_bnorm, dim3(nb), dim3(kBT), 0, s, S, rhs, G.part, G.P);
  hipLaunchKernelGGL(k_bgm_init, dim3(count), dim3(kBT), 0, s, S, G, o->rtol);
  hipLaunchKernelGGL(k_bscale, dim3(nb), dim3(kBT), 0, s, S, (const double*)x, (const double*)G.sc, x);
  if ((rc = W.check("batch set-up"))) return rc;

  // multigrid: every instance's hierarchy set up as mns_solve does; its
  // level-0 operator (the instance's, or its Picard copy) and that level's
  // lambda_max; a batch over the level-0 operators for this call when one of
  // them is a copy
  struct FineGuard {
    mns_batch* B;
    hipStream_t s;
    BatchMG* bmg = nullptr;
    ~FineGuard() {
      if (B->mg_fine || bmg) (void)hipStreamSynchronize(s);  // graph replays may still read their tables
      bmg_free(bmg);
      if (B->mg_fine) mns_batch_destroy(B->mg_fine);
      B->mg_fine = nullptr;
      B->mg_fine_hs.clear();
    }
  } fine_guard{B, s};
  std::vector<double> lam0(count, 0.0);
  if (mgp) {
    B->mg_fine_hs.assign(count, nullptr);
    bool copies = false;
    for (int i = 0; i < count; ++i) {
      if ((rc = mg_instance_setup(B->hs[i], o, s, &B->mg_fine_hs[i], &lam0[i])))
        return W.fail(rc, "batch multigrid, instance " + std::to_string(i) + ": " + B->hs[i]->err);
      copies = copies || B->mg_fine_hs[i] != B->hs[i];
    }
    if (copies) {
      if ((rc = mns_batch_create(B->mg_fine_hs.data(), count, &B->mg_fine)))
        return W.fail(rc, "batch of the level-0 operators: " + B->mg_fine_hs[0]->err);
      W.F = B->mg_fine;
    } else {
      W.F = B;
    }
    // the coarse levels batched when every hierarchy ends in a direct solve
    rc = bmg_setup(B, B->mg_fine_hs.data(), o, o->precond == MNS_PRECOND_MG, s, &fine_guard.bmg);
    if (rc && rc != MNS_ERR_UNSUPPORTED) return W.fail(rc, B->err);
    W.bmg = fine_guard.bmg;
  }
  // diagonals of every instance (Alg. Alg-diagonal), FP64 and FP32: each
  // handle's cached diagonal, computed when its linearization changed (with
  // multigrid: the diagonal of the level-0 operator, set up by its hierarchy)
  for (int i = 0; i < count; ++i) {
    mns_handle* h = mgp ? B->mg_fine_hs[i] : B->hs[i];
    if (!mgp && (rc = cached_diagonal(h, s))) return W.fail(rc, "batch diagonal: " + h->err);
    if ((e = hipMemcpyAsync(W.diag64 + B->offsets[i], h->d_diag64, (size_t)h->ndofs * sizeof(double),
                            hipMemcpyDeviceToDevice, s)) != hipSuccess ||
        (e = hipMemcpyAsync(W.diag32 + B->offsets[i], h->d_diag32, (size_t)h->ndofs * sizeof(float),
                            hipMemcpyDeviceToDevice, s)) != hipSuccess)
      return W.fail(MNS_ERR_HIP, std::string("batch diagonal copy: ") + hipGetErrorString(e));
  }

  if (mgp) {
    // the level-0 lambda_max of every hierarchy, then the smoother's scalars
    for (int i = 0; i < count; ++i)
      if ((e = hipMemcpyAsync(G.inst + (size_t)i * BI_N + BI_LAM, &lam0[i], sizeof(double), hipMemcpyHostToDevice,
                              s)) != hipSuccess)
        return W.fail(MNS_ERR_HIP, std::string("batch multigrid lambda: ") + hipGetErrorString(e));
    hipLaunchKernelGGL(k_bcheb_coef, dim3(1), dim3(kBT), 0, s, G, o->mg_smooth_degree, o->cheb_lambda_factor,
                       o->mg_smooth_range);
    if ((e = hipStreamSynchronize(s)) != hipSuccess)
      return W.fail(MNS_ERR_HIP, std::string("batch multigrid set-up: ") + hipGetErrorString(e));
  } else if (o->precond != -1) {
    // lambda_max of D^-1 J per instance by power iteration from the constant
    // vector, then the Chebyshev scalars, all on the device
    if ((rc = launch_fill<double>(W.t, 1.0, N, s))) return W.fail(rc, "fill");
    hipLaunchKernelGGL(k_bpower_start, dim3(1), dim3(kBT), 0, s, S, G);
    hipLaunchKernelGGL(k_bscale, dim3(nb), dim3(kBT), 0, s, S, (const double*)W.t, (const double*)G.sc, W.cb);
    for (int it = 0; it < o->eig_iters; ++it) {
      if ((rc = W.jac64(W.cb, W.t, s))) return rc;
      hipLaunchKernelGGL(k_bpower, dim3(nb), dim3(kBT), 0, s, S, (const double*)W.t, (const double*)W.diag64, W.cb,
                         G.part, G.P);
      hipLaunchKernelGGL(k_bpower_norm, dim3(count), dim3(kBT), 0, s, S, G);
      hipLaunchKernelGGL(k_bscale, dim3(nb), dim3(kBT), 0, s, S, (const double*)W.cb, (const double*)G.sc, W.cb);
    }
    hipLaunchKernelGGL(k_bcheb_coef, dim3(1), dim3(kBT), 0, s, G, o->cheb_degree, o->cheb_lambda_factor,
                       o->cheb_range);
    if ((rc = W.check("batch power iteration"))) return rc;
  }

  int total = 0;
  while (total < o->maxit) {
    // true residuals; converged instances stop
    if ((rc = W.jac64(x, W.t, s))) return rc;
    hipLaunchKernelGGL(k_bresid, dim3(nb), dim3(kBT), 0, s, S, rhs, (const double*)W.t, W.r, G.part, G.P);
    hipLaunchKernelGGL(k_bgm_cycle, dim3(count), dim3(kBT), 0, s, S, G);
    hipLaunchKernelGGL(k_bgm_flags, dim3(1), dim3(kBT), 0, s, G, 1);
    hipLaunchKernelGGL(k_bgm_next, dim3(nb), dim3(kBT), 0, s, S, G, W.V, N, (const double*)W.r);
    if ((rc = W.check("batch cycle start")) || (rc = W.read_state())) return rc;
    if (W.misc(BG_BROKEN) != 0.0) return W.fail(MNS_ERR_HIP, "non-finite value in the batched power iteration");
    if (W.misc(BG_ALLDONE) != 0.0) break;
    // iterations in chunks between readbacks; the chunk follows the observed
    // convergence rate of the slowest instance (iterations past convergence
    // leave the state unchanged)
    const int cycle = std::min(m, o->maxit - total);
    int launched = 0, jj = 0;
    double worst0 = W.misc(BG_WORST), worst = worst0;
    while (launched < cycle) {
      int chunk = 1;
      if (jj > 0 && worst < worst0 && worst > 1.0) {
        const double rate = std::log(worst / worst0) / jj;  // < 0
        const double left = std::log(1.0 / worst) / rate;
        chunk = (int)std::max(1.0, std::min(8.0, std::floor(0.5 * left)));
      }
      chunk = std::min(chunk, cycle - launched);
      if ((rc = W.iterations(chunk))) return rc;
      launched += chunk;
      if ((rc = W.read_state())) return rc;
      if (W.misc(BG_BROKEN) != 0.0) return W.fail(MNS_ERR_HIP, "non-finite value in batched FGMRES");
      jj = (int)W.misc(BG_J);
      worst = W.misc(BG_WORST);
      if (W.misc(BG_ALLDONE) != 0.0) break;
    }
    if (jj < 1) return W.fail(MNS_ERR_HIP, "batched FGMRES cycle made no progress");
    total += jj;
    W.vm64 += jj * W.it_vm64;
    W.vm32 += jj * W.it_vm32;
    // x_i += Z y_i with y_i = H_i^-1 g_i
    hipLaunchKernelGGL(k_bgm_backsub, dim3(1), dim3(kBT), 0, s, G);
    hipLaunchKernelGGL(k_bgm_update, dim3(nb), dim3(kBT), 0, s, S, G, (const double*)W.Z, N, x);
    if ((rc = W.check("batch solution update"))) return rc;
  }
  // final true residuals
  if ((rc = W.jac64(x, W.t, s))) return rc;
  hipLaunchKernelGGL(k_bresid, dim3(nb), dim3(kBT), 0, s, S, rhs, (const double*)W.t, W.r, G.part, G.P);
  hipLaunchKernelGGL(k_bgm_final, dim3(count), dim3(kBT), 0, s, S, G);
  if ((rc = W.check("batch residual")) || (rc = W.read_state())) return rc;
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  bool all = true;
  for (int i = 0; i < count; ++i) {
    const double r2 = W.inst(i, BI_RES), bn = W.inst(i, BI_BN);
    const bool ok = r2 <= W.inst(i, BI_TARGET);
    all = all && ok;
    if (reps) {
      mns_solve_report& R = reps[i];
      R = mns_solve_report{};
      R.iterations = (int)W.inst(i, BI_ITS);
      R.status = ok ? MNS_OK : MNS_ERR_NOT_CONVERGED;
      R.rel_residual = bn > 0 ? r2 / bn : 0.0;
      R.lambda_max = o->precond != -1 ? W.inst(i, BI_LAM) : 0.0;
      R.seconds = secs;
      R.vmults_f64 = W.vm64;
      R.vmults_f32 = W.vm32;
    }
  }
  if (!all) return W.fail(MNS_ERR_NOT_CONVERGED, "batched FGMRES reached maxit for some instances");
  return MNS_OK;
}

}  // namespace mns
