// Batched FGMRES: the instances of a batch solve J_i x_i = b_i together, in
// lockstep, every iteration one batched preconditioner application, one
// batched FP64 Jacobian application and batched Gram-Schmidt reductions over
// the concatenated vectors.  The arithmetic of each instance is that of
// mns_solve with the Jacobi-Chebyshev preconditioner (Sec. 3.4 smoother
// polynomial with the diagonal of Alg. Alg-diagonal); only the reduction
// order of the dot products differs.  Vector kernels work on blocks that never
// straddle two instances, so per-instance scalars are read once per block.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "mns_internal.hpp"

namespace mns {
namespace {

constexpr int kBT = 256;           // threads per block
constexpr int kBChunk = kBT * 8;   // vector entries per block
constexpr int kBK = 32;            // register width of the dot kernels (restart <= 31)

struct BSeg {
  const long long* bstart;  // first block of each instance (count + 1)
  const long long* off;     // first entry of each instance (count + 1)
  int count;
};

__device__ inline void bseg_range(const BSeg& S, long long b, int& i, long long& lo, long long& hi) {
  int a = 0, z = S.count - 1;  // last instance whose first block is at or before b
  while (a < z) {
    const int mid = (a + z + 1) >> 1;
    if (S.bstart[mid] <= b) a = mid;
    else z = mid - 1;
  }
  i = a;
  lo = S.off[a] + (b - S.bstart[a]) * kBChunk;
  hi = lo + kBChunk < S.off[a + 1] ? lo + kBChunk : S.off[a + 1];
}

// per-block sums of K thread values into part[blockIdx.x * K + k]
template <int MAXK>
__device__ inline void bsum_store(double (&v)[MAXK], int K, double* part) {
  __shared__ double red[kBT / 64][MAXK];
  const int lane = threadIdx.x % 64, wid = threadIdx.x / 64;
#pragma unroll
  for (int k = 0; k < MAXK; ++k) {
    if (k < K) {
      double x = v[k];
      for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
      if (lane == 0) red[wid][k] = x;
    }
  }
  __syncthreads();
  if ((int)threadIdx.x < K) {
    double t = 0;
    for (int w = 0; w < kBT / 64; ++w) t += red[w][threadIdx.x];
    part[(long long)blockIdx.x * K + threadIdx.x] = t;
  }
}

// dots of w with V_0 .. V_{K-1} (stride N) and, with self, w . w (entry K)
__global__ __launch_bounds__(kBT) void k_bdots(BSeg S, const double* __restrict__ V, long long N, int K,
                                               const double* __restrict__ w, int self, double* __restrict__ part) {
  int i;
  long long lo, hi;
  bseg_range(S, blockIdx.x, i, lo, hi);
  double acc[kBK];
#pragma unroll
  for (int k = 0; k < kBK; ++k) acc[k] = 0;
  for (long long r = lo + threadIdx.x; r < hi; r += kBT) {
    const double wr = w[r];
#pragma unroll
    for (int k = 0; k < kBK; ++k) {
      if (k < K) acc[k] += V[(long long)k * N + r] * wr;
      if (self && k == K) acc[k] += wr * wr;
    }
  }
  bsum_store<kBK>(acc, K + self, part);
}

// out[i * Kp + k] = sum of the partial sums of instance i's blocks (fixed order)
__global__ __launch_bounds__(kBT) void k_bsum(BSeg S, const double* __restrict__ part, int Kp,
                                              double* __restrict__ out) {
  __shared__ double red[kBT];
  const int i = blockIdx.x;
  const long long b0 = S.bstart[i], b1 = S.bstart[i + 1];
  for (int k = 0; k < Kp; ++k) {
    double t = 0;
    for (long long b = b0 + threadIdx.x; b < b1; b += kBT) t += part[b * Kp + k];
    red[threadIdx.x] = t;
    __syncthreads();
    for (int off = kBT / 2; off > 0; off >>= 1) {
      if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[(long long)i * Kp + k] = red[0];
    __syncthreads();
  }
}

// w -= sum_k h[i][k] V_k (h: count x K); with dots, then the dots of the new
// w with V_k (entries 0..K-1) and w . w (entry K), else w . w only
__global__ __launch_bounds__(kBT) void k_baxpy(BSeg S, const double* __restrict__ V, long long N, int K,
                                               const double* __restrict__ h, double* __restrict__ w, int dots,
                                               double* __restrict__ part) {
  int i;
  long long lo, hi;
  bseg_range(S, blockIdx.x, i, lo, hi);
  double hh[kBK], acc[kBK];
#pragma unroll
  for (int k = 0; k < kBK; ++k) {
    hh[k] = 0;
    if (k < K) hh[k] = h[(long long)i * K + k];
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
    if (dots) {
#pragma unroll
      for (int k = 0; k < kBK; ++k) {
        if (k < K) acc[k] += v[k] * x;
        if (k == K) acc[k] += x * x;
      }
    } else {
      acc[0] += x * x;
    }
  }
  bsum_store<kBK>(acc, dots ? K + 1 : 1, part);
}

// y = s[i] x; x and y may be the same vector
__global__ __launch_bounds__(kBT) void k_bscale(BSeg S, const double* x, const double* __restrict__ sc, double* y) {
  int i;
  long long lo, hi;
  bseg_range(S, blockIdx.x, i, lo, hi);
  const double a = sc[i];
  for (long long r = lo + threadIdx.x; r < hi; r += kBT) y[r] = a * x[r];
}

// x += sum_k y[i][k] Z_k (y: count x K)
__global__ __launch_bounds__(kBT) void k_bupdate(BSeg S, const double* __restrict__ Z, long long N, int K,
                                                 const double* __restrict__ y, double* __restrict__ x) {
  int i;
  long long lo, hi;
  bseg_range(S, blockIdx.x, i, lo, hi);
  for (long long r = lo + threadIdx.x; r < hi; r += kBT) {
    double a = x[r];
    for (int k = 0; k < K; ++k) a += y[(long long)i * K + k] * Z[(long long)k * N + r];
    x[r] = a;
  }
}

// r = b - t, partial ||r||^2
__global__ __launch_bounds__(kBT) void k_bresid(BSeg S, const double* __restrict__ b, const double* __restrict__ t,
                                                double* __restrict__ r, double* __restrict__ part) {
  int i;
  long long lo, hi;
  bseg_range(S, blockIdx.x, i, lo, hi);
  double acc[1] = {0};
  for (long long q = lo + threadIdx.x; q < hi; q += kBT) {
    const double v = b[q] - t[q];
    r[q] = v;
    acc[0] += v * v;
  }
  bsum_store<1>(acc, 1, part);
}

// y = D^-1 t (power iteration), partial ||y||^2
__global__ __launch_bounds__(kBT) void k_bpower(BSeg S, const double* __restrict__ t, const double* __restrict__ diag,
                                                double* __restrict__ y, double* __restrict__ part) {
  int i;
  long long lo, hi;
  bseg_range(S, blockIdx.x, i, lo, hi);
  double acc[1] = {0};
  for (long long q = lo + threadIdx.x; q < hi; q += kBT) {
    const double v = t[q] / diag[q];
    y[q] = v;
    acc[0] += v * v;
  }
  bsum_store<1>(acc, 1, part);
}

// Chebyshev polynomial of D^-1 J with per-instance scalars: start
// (inv_theta[i]) and step k (c[k][i][0..1])
template <typename Real>
__global__ __launch_bounds__(kBT) void k_bcheb_init(BSeg S, const Real* __restrict__ b, const Real* __restrict__ diag,
                                                    const double* __restrict__ inv_theta, Real* __restrict__ r,
                                                    Real* __restrict__ d, Real* __restrict__ x) {
  int i;
  long long lo, hi;
  bseg_range(S, blockIdx.x, i, lo, hi);
  const Real it = (Real)inv_theta[i];
  for (long long q = lo + threadIdx.x; q < hi; q += kBT) {
    const Real bi = b[q];
    const Real di = it * bi / diag[q];
    r[q] = bi;
    d[q] = di;
    x[q] = di;
  }
}

template <typename Real>
__global__ __launch_bounds__(kBT) void k_bcheb_step(BSeg S, Real* __restrict__ r, const Real* __restrict__ Jd,
                                                    const Real* __restrict__ diag, const double* __restrict__ c,
                                                    Real* __restrict__ d, Real* __restrict__ x) {
  int i;
  long long lo, hi;
  bseg_range(S, blockIdx.x, i, lo, hi);
  const Real c1 = (Real)c[2 * i], c2 = (Real)c[2 * i + 1];
  for (long long q = lo + threadIdx.x; q < hi; q += kBT) {
    const Real ri = r[q] - Jd[q];
    const Real di = c1 * d[q] + c2 * ri / diag[q];
    r[q] = ri;
    d[q] = di;
    x[q] += di;
  }
}

struct BatchSolver {
  mns_batch* B;
  hipStream_t s;
  int count, m;
  long long N, nblk;
  BSeg S;
  double *V, *Z, *w, *r, *t, *diag64, *cb, *cx, *cr, *cd, *ct;
  float *b32, *x32, *r32, *d32, *t32, *diag32;
  double *part, *out, *coef;  // device small buffers
  double *h_out, *h_coef;     // pinned mirrors
  int vm64 = 0, vm32 = 0;

  int fail(int code, const std::string& msg) {
    B->err = msg;
    return code;
  }
  int check(const char* what) {
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? MNS_OK : fail(MNS_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
  }
  // per-instance sums (count x Kp) of the last partial sums -> host
  int sums(int Kp, std::vector<double>& host) {
    hipLaunchKernelGGL(k_bsum, dim3(count), dim3(kBT), 0, s, S, part, Kp, out);
    hipError_t e = hipMemcpyAsync(h_out, out, (size_t)count * Kp * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(MNS_ERR_HIP, std::string("batch readback: ") + hipGetErrorString(e));
    host.assign(h_out, h_out + (size_t)count * Kp);
    return MNS_OK;
  }
  // host values (count x K) -> coef on the device; the staging buffer is
  // reused only after a later synchronization
  int upload(const std::vector<double>& v) {
    std::memcpy(h_coef, v.data(), v.size() * sizeof(double));
    hipError_t e = hipMemcpyAsync(coef, h_coef, v.size() * sizeof(double), hipMemcpyHostToDevice, s);
    return e == hipSuccess ? MNS_OK : fail(MNS_ERR_HIP, std::string("batch upload: ") + hipGetErrorString(e));
  }
  int jac64(const double* src, double* dst) {
    ++vm64;
    return launch_batch_jacobian<double>(B, src, dst, s);
  }
  int jac32(const float* src, float* dst) {
    ++vm32;
    return launch_batch_jacobian<float>(B, src, dst, s);
  }
  int scale(const double* x, const std::vector<double>& sc, double* y) {
    int rc = upload(sc);
    if (rc) return rc;
    hipLaunchKernelGGL(k_bscale, dim3((unsigned)nblk), dim3(kBT), 0, s, S, x, coef, y);
    return check("batch scale");
  }
};

}  // namespace

void batch_solver_free(mns_batch* b) {
  if (b->d_seg) (void)hipFree(b->d_seg);
  if (b->ws) (void)hipFree(b->ws);
  if (b->ws32) (void)hipFree(b->ws32);
  if (b->d_small) (void)hipFree(b->d_small);
  if (b->h_small) (void)hipHostFree(b->h_small);
  b->d_seg = nullptr;
  b->ws = nullptr;
  b->ws32 = nullptr;
  b->d_small = nullptr;
  b->h_small = nullptr;
  b->ws_m = 0;
}

int batch_solve_impl(mns_batch* B, const double* rhs, double* x, const mns_solve_opts* o, mns_solve_report* reps,
                     hipStream_t s) {
  const auto t0 = std::chrono::steady_clock::now();
  const int count = (int)B->hs.size();
  const long long N = B->ndofs;
  const int m = o->restart;
  hipError_t e;
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
    const size_t small = (size_t)B->nvblk * (kBK + 1) + (size_t)count * (kBK + 1) * 2 + 64 * (size_t)count;
    if ((e = hipMalloc((void**)&B->d_small, small * sizeof(double))) != hipSuccess ||
        (e = hipHostMalloc((void**)&B->h_small, (size_t)count * (kBK + 1) * 2 * sizeof(double) + 64 * (size_t)count *
                                                    sizeof(double), hipHostMallocDefault)) != hipSuccess) {
      B->err = std::string("batch buffers: ") + hipGetErrorString(e);
      return MNS_ERR_HIP;
    }
  }
  if (B->ws_m < m) {
    if (B->ws) (void)hipFree(B->ws);
    if (B->ws32) (void)hipFree(B->ws32);
    B->ws = nullptr;
    B->ws32 = nullptr;
    B->ws_m = 0;
    if ((e = hipMalloc((void**)&B->ws, (size_t)(2 * m + 10) * N * sizeof(double))) != hipSuccess ||
        (e = hipMalloc((void**)&B->ws32, 6 * (size_t)N * sizeof(float))) != hipSuccess) {
      B->err = std::string("hipMalloc batch workspace: ") + hipGetErrorString(e);
      return MNS_ERR_HIP;
    }
    B->ws_m = m;
  }
  BatchSolver W;
  W.B = B;
  W.s = s;
  W.count = count;
  W.m = m;
  W.N = N;
  W.nblk = B->nvblk;
  W.S = BSeg{B->d_seg, B->d_seg + count + 1, count};
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
  W.b32 = B->ws32;
  W.x32 = W.b32 + N;
  W.r32 = W.x32 + N;
  W.d32 = W.r32 + N;
  W.t32 = W.d32 + N;
  W.diag32 = W.t32 + N;
  W.part = B->d_small;
  W.out = W.part + (size_t)W.nblk * (kBK + 1);
  W.coef = W.out + (size_t)count * (kBK + 1);
  W.h_out = B->h_small;
  W.h_coef = W.h_out + (size_t)count * (kBK + 1);
  const unsigned nb = (unsigned)W.nblk;
  int rc;

  // diagonals of every instance (Alg. Alg-diagonal), FP64 and FP32
  for (int i = 0; i < count; ++i)
    if ((rc = launch_diagonal<double>(B->hs[i], W.diag64 + B->offsets[i], s)))
      return W.fail(rc, "batch diagonal: " + B->hs[i]->err);
  if ((rc = launch_cast_f64_f32(W.diag64, W.diag32, N, s))) return W.fail(rc, "cast");

  std::vector<double> sums, sc(count);
  // spectra: power iteration of D^-1 J per instance from the constant vector
  std::vector<double> lam(count, 1.0);
  if (o->precond != -1) {
    if ((rc = launch_fill<double>(W.t, 1.0, N, s))) return W.fail(rc, "fill");
    for (int i = 0; i < count; ++i) sc[i] = 1.0 / std::sqrt((double)B->hs[i]->ndofs);
    if ((rc = W.scale(W.t, sc, W.cb))) return rc;
    for (int it = 0; it < o->eig_iters; ++it) {
      if ((rc = W.jac64(W.cb, W.t))) return rc;
      hipLaunchKernelGGL(k_bpower, dim3(nb), dim3(kBT), 0, s, W.S, W.t, W.diag64, W.cb, W.part);
      if ((rc = W.check("power step")) || (rc = W.sums(1, sums))) return rc;
      for (int i = 0; i < count; ++i) {
        lam[i] = std::sqrt(sums[i]);
        if (!(lam[i] > 0) || !std::isfinite(lam[i])) return W.fail(MNS_ERR_HIP, "batch power iteration broke down");
        sc[i] = 1.0 / lam[i];
      }
      if ((rc = W.scale(W.cb, sc, W.cb))) return rc;
    }
  }
  // Chebyshev scalars per instance: start 1/theta, step k (c1, c2)
  const int deg = o->cheb_degree;
  std::vector<double> inv_theta(count), cheb((size_t)deg * count * 2);
  for (int i = 0; i < count; ++i) {
    const double beta = lam[i] * o->cheb_lambda_factor, alpha = beta / o->cheb_range;
    const double theta = 0.5 * (beta + alpha), delta = 0.5 * (beta - alpha), sigma = theta / delta;
    inv_theta[i] = 1.0 / theta;
    double rho = 1.0 / sigma;
    for (int k = 0; k < deg; ++k) {
      const double rn = 1.0 / (2.0 * sigma - rho);
      cheb[((size_t)k * count + i) * 2] = rn * rho;
      cheb[((size_t)k * count + i) * 2 + 1] = 2.0 * rn / delta;
      rho = rn;
    }
  }
  // the Chebyshev scalars stay on the device after the coefficient area
  double* d_cheb = W.coef + (size_t)count * kBK;
  double* d_inv_theta = d_cheb + (size_t)deg * count * 2;
  {
    std::vector<double> all(cheb);
    all.insert(all.end(), inv_theta.begin(), inv_theta.end());
    if (2 * deg + 1 > 65) return W.fail(MNS_ERR_INVALID_ARG, "Chebyshev degree above 32 in the batched solver");
    if ((e = hipMemcpyAsync(d_cheb, all.data(), all.size() * sizeof(double), hipMemcpyHostToDevice, s)) !=
            hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
      return W.fail(MNS_ERR_HIP, std::string("batch upload: ") + hipGetErrorString(e));
  }
  // z = M^-1 v for every instance
  auto precondition = [&](const double* v, double* z) -> int {
    if (o->precond == -1) {
      const hipError_t e2 = hipMemcpyAsync(z, v, (size_t)N * sizeof(double), hipMemcpyDeviceToDevice, s);
      return e2 == hipSuccess ? MNS_OK : W.fail(MNS_ERR_HIP, "batch copy");
    }
    int rc2;
    if (o->precond == MNS_F64) {
      hipLaunchKernelGGL(k_bcheb_init<double>, dim3(nb), dim3(kBT), 0, s, W.S, v, W.diag64, d_inv_theta, W.cr, W.cd,
                         z);
      for (int k = 0; k < deg; ++k) {
        if ((rc2 = W.jac64(W.cd, W.ct))) return rc2;
        hipLaunchKernelGGL(k_bcheb_step<double>, dim3(nb), dim3(kBT), 0, s, W.S, W.cr, W.ct, W.diag64,
                           d_cheb + (size_t)k * count * 2, W.cd, z);
      }
      return W.check("batch Chebyshev");
    }
    if ((rc2 = launch_cast_f64_f32(v, W.b32, N, s))) return W.fail(rc2, "cast");
    hipLaunchKernelGGL(k_bcheb_init<float>, dim3(nb), dim3(kBT), 0, s, W.S, W.b32, W.diag32, d_inv_theta, W.r32, W.d32,
                       W.x32);
    for (int k = 0; k < deg; ++k) {
      if ((rc2 = W.jac32(W.d32, W.t32))) return rc2;
      hipLaunchKernelGGL(k_bcheb_step<float>, dim3(nb), dim3(kBT), 0, s, W.S, W.r32, W.t32, W.diag32,
                         d_cheb + (size_t)k * count * 2, W.d32, W.x32);
    }
    if ((rc2 = launch_cast_f32_f64(W.x32, z, N, s))) return W.fail(rc2, "cast");
    return W.check("batch Chebyshev");
  };

  // ||b_i||
  hipLaunchKernelGGL(k_bdots, dim3(nb), dim3(kBT), 0, s, W.S, rhs, N, 1, rhs, 0, W.part);
  if ((rc = W.check("batch norm")) || (rc = W.sums(1, sums))) return rc;
  std::vector<double> bn(count), target(count), rn(count, 0.0);
  std::vector<int> its(count, 0), conv(count, 0);
  for (int i = 0; i < count; ++i) {
    bn[i] = std::sqrt(sums[i]);
    target[i] = o->rtol * bn[i];
    sc[i] = bn[i] > 0 ? 1.0 : 0.0;  // zero right-hand side: x = 0
  }
  if ((rc = W.scale(x, sc, x))) return rc;

  std::vector<double> H((size_t)count * (m + 1) * m), cs((size_t)count * m), sn((size_t)count * m),
      g((size_t)count * (m + 1)), hc((size_t)count * (m + 1)), y;
  int total = 0;
  while (total < o->maxit) {
    // true residuals; converged instances stop
    if ((rc = W.jac64(x, W.t))) return rc;
    hipLaunchKernelGGL(k_bresid, dim3(nb), dim3(kBT), 0, s, W.S, rhs, W.t, W.r, W.part);
    if ((rc = W.check("batch residual")) || (rc = W.sums(1, sums))) return rc;
    bool any = false;
    std::vector<int> active(count, 0), done(count, 1), jn(count, 0);
    for (int i = 0; i < count; ++i) {
      rn[i] = std::sqrt(sums[i]);
      conv[i] = rn[i] <= target[i];
      active[i] = !conv[i];
      done[i] = conv[i];
      any = any || active[i];
      sc[i] = active[i] ? 1.0 / rn[i] : 0.0;
    }
    if (!any) break;
    if ((rc = W.scale(W.r, sc, W.V))) return rc;
    std::fill(g.begin(), g.end(), 0.0);
    for (int i = 0; i < count; ++i) g[(size_t)i * (m + 1)] = active[i] ? rn[i] : 0.0;
    int j = 0;
    for (; j < m && total < o->maxit; ++j, ++total) {
      double* Vj = W.V + (size_t)j * N;
      double* Zj = W.Z + (size_t)j * N;
      if ((rc = precondition(Vj, Zj))) return rc;
      if ((rc = W.jac64(Zj, W.w))) return rc;
      const int K = j + 1;
      // (1) h = V^T w and w . w; (2) w -= V h with h2 = V^T w and w . w;
      // (3) where the norm dropped below 0.7 of its value, w -= V h2
      hipLaunchKernelGGL(k_bdots, dim3(nb), dim3(kBT), 0, s, W.S, W.V, N, K, W.w, 1, W.part);
      if ((rc = W.check("batch dots")) || (rc = W.sums(K + 1, sums))) return rc;
      std::vector<double> h1((size_t)count * K), wn0(count);
      for (int i = 0; i < count; ++i) {
        for (int k = 0; k < K; ++k) h1[(size_t)i * K + k] = sums[(size_t)i * (K + 1) + k];
        wn0[i] = std::sqrt(sums[(size_t)i * (K + 1) + K]);
      }
      if ((rc = W.upload(h1))) return rc;
      hipLaunchKernelGGL(k_baxpy, dim3(nb), dim3(kBT), 0, s, W.S, W.V, N, K, W.coef, W.w, 1, W.part);
      if ((rc = W.check("batch update")) || (rc = W.sums(K + 1, sums))) return rc;
      std::vector<double> h2((size_t)count * K, 0.0), wn(count);
      bool reorth = false;
      for (int i = 0; i < count; ++i) {
        wn[i] = std::sqrt(sums[(size_t)i * (K + 1) + K]);
        if (wn[i] < 0.7 * wn0[i]) {
          reorth = true;
          for (int k = 0; k < K; ++k) h2[(size_t)i * K + k] = sums[(size_t)i * (K + 1) + k];
        }
      }
      if (reorth) {
        if ((rc = W.upload(h2))) return rc;
        hipLaunchKernelGGL(k_baxpy, dim3(nb), dim3(kBT), 0, s, W.S, W.V, N, K, W.coef, W.w, 0, W.part);
        if ((rc = W.check("batch update")) || (rc = W.sums(1, sums))) return rc;
        for (int i = 0; i < count; ++i) wn[i] = std::sqrt(sums[i]);
      }
      bool all_done = true;
      for (int i = 0; i < count; ++i) {
        sc[i] = 0.0;
        if (done[i]) continue;
        double* hcol = &hc[(size_t)i * (m + 1)];
        for (int k = 0; k < K; ++k) hcol[k] = h1[(size_t)i * K + k] + h2[(size_t)i * K + k];
        hcol[K] = wn[i];
        if (!std::isfinite(wn[i])) return W.fail(MNS_ERR_HIP, "non-finite value in batched FGMRES");
        double* csi = &cs[(size_t)i * m];
        double* sni = &sn[(size_t)i * m];
        double* gi = &g[(size_t)i * (m + 1)];
        for (int k = 0; k < j; ++k) {
          const double a = csi[k] * hcol[k] + sni[k] * hcol[k + 1];
          const double b2 = -sni[k] * hcol[k] + csi[k] * hcol[k + 1];
          hcol[k] = a;
          hcol[k + 1] = b2;
        }
        const double den = std::hypot(hcol[j], hcol[j + 1]);
        csi[j] = den > 0 ? hcol[j] / den : 1.0;
        sni[j] = den > 0 ? hcol[j + 1] / den : 0.0;
        hcol[j] = den;
        hcol[j + 1] = 0.0;
        gi[j + 1] = -sni[j] * gi[j];
        gi[j] = csi[j] * gi[j];
        for (int k = 0; k <= j; ++k) H[((size_t)i * (m + 1) + k) * m + j] = hcol[k];
        jn[i] = j + 1;
        ++its[i];
        if (std::fabs(gi[j + 1]) <= target[i] || wn[i] == 0) done[i] = 1;
        else sc[i] = 1.0 / wn[i];
        all_done = all_done && done[i];
      }
      if (j + 1 < m && !all_done && (rc = W.scale(W.w, sc, W.V + (size_t)(j + 1) * N))) return rc;
      if (all_done) {
        ++j;
        ++total;
        break;
      }
    }
    // x_i += Z y_i with y_i = H_i^-1 g_i (upper triangular, order jn[i])
    const int Kmax = std::max(1, j);
    y.assign((size_t)count * Kmax, 0.0);
    for (int i = 0; i < count; ++i) {
      const int ji = active[i] ? jn[i] : 0;
      for (int a = ji - 1; a >= 0; --a) {
        double sum = g[(size_t)i * (m + 1) + a];
        for (int k2 = a + 1; k2 < ji; ++k2) sum -= H[((size_t)i * (m + 1) + a) * m + k2] * y[(size_t)i * Kmax + k2];
        const double d = H[((size_t)i * (m + 1) + a) * m + a];
        y[(size_t)i * Kmax + a] = d != 0 ? sum / d : 0.0;
      }
    }
    if ((rc = W.upload(y))) return rc;
    hipLaunchKernelGGL(k_bupdate, dim3(nb), dim3(kBT), 0, s, W.S, W.Z, N, Kmax, W.coef, x);
    if ((rc = W.check("batch solution update"))) return rc;
    (void)hipStreamSynchronize(s);  // the staging buffer is reused by the next cycle
  }
  // final true residuals
  if ((rc = W.jac64(x, W.t))) return rc;
  hipLaunchKernelGGL(k_bresid, dim3(nb), dim3(kBT), 0, s, W.S, rhs, W.t, W.r, W.part);
  if ((rc = W.check("batch residual")) || (rc = W.sums(1, sums))) return rc;
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  bool all = true;
  for (int i = 0; i < count; ++i) {
    const double r2 = std::sqrt(sums[i]);
    const bool ok = r2 <= target[i];
    all = all && ok;
    if (reps) {
      mns_solve_report& R = reps[i];
      R = mns_solve_report{};
      R.iterations = its[i];
      R.status = ok ? MNS_OK : MNS_ERR_NOT_CONVERGED;
      R.rel_residual = bn[i] > 0 ? r2 / bn[i] : 0.0;
      R.lambda_max = lam[i];
      R.seconds = secs;
      R.vmults_f64 = W.vm64;
      R.vmults_f32 = W.vm32;
    }
  }
  if (!all) return W.fail(MNS_ERR_NOT_CONVERGED, "batched FGMRES reached maxit for some instances");
  return MNS_OK;
}

}  // namespace mns
