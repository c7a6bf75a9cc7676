// Flexible GMRES(m) in FP64 with a Jacobi-Chebyshev polynomial preconditioner
// whose Jacobian applications run in FP32 (mixed) or FP64 (plain).  The outer
// Krylov basis, the Hessenberg reduction and the true residual are FP64.
//
// Orthogonalization: classical Gram-Schmidt with one reorthogonalization pass
// when the projected norm drops below 0.7 of the original (DGKS criterion);
// each pass is one fused multi-dot kernel and one fused multi-axpy/norm kernel
// with a deterministic two-stage reduction.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "mns_internal.hpp"

namespace mns {

constexpr int kRedBlocks = 1024;  // partial-sum blocks of the reductions
constexpr int kRedThreads = 256;

template <typename From, typename To>
__global__ void k_cast(const From* __restrict__ a, To* __restrict__ b, long long n) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) b[i] = (To)a[i];
}

// block-level sum of K values per thread into out[blockIdx.x * K + i]
template <int MAXK>
__device__ inline void block_sum_store(double (&v)[MAXK], int K, double* out) {
  __shared__ double s[kRedThreads / 64][MAXK];
  const int lane = threadIdx.x % 64, wid = threadIdx.x / 64;
  for (int i = 0; i < K; ++i) {
    double x = v[i];
    for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
    if (lane == 0) s[wid][i] = x;
  }
  __syncthreads();
  if (threadIdx.x < K) {
    double t = 0;
    for (int w = 0; w < kRedThreads / 64; ++w) t += s[w][threadIdx.x];
    out[blockIdx.x * K + threadIdx.x] = t;
  }
}

// partial dots of w with V_0 .. V_{K-1} (contiguous, stride n), K <= 32 per launch
__global__ __launch_bounds__(kRedThreads) void k_multidot(const double* __restrict__ V, long long n, int K,
                                                          const double* __restrict__ w, double* __restrict__ part) {
  double acc[32];
  for (int i = 0; i < 32; ++i) acc[i] = 0;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += stride) {
    const double wr = w[r];
#pragma unroll 4
    for (int i = 0; i < K; ++i) acc[i] += V[(long long)i * n + r] * wr;
  }
  block_sum_store<32>(acc, K, part);
}

// w -= sum_i h_i V_i ; partial ||w||^2
__global__ __launch_bounds__(kRedThreads) void k_multiaxpy_norm(const double* __restrict__ V, long long n, int K,
                                                                const double* __restrict__ hcoef,
                                                                double* __restrict__ w, double* __restrict__ part) {
  double acc[1] = {0};
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += stride) {
    double x = w[r];
    for (int i = 0; i < K; ++i) x -= hcoef[i] * V[(long long)i * n + r];
    w[r] = x;
    acc[0] += x * x;
  }
  block_sum_store<1>(acc, 1, part);
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
                            Real* __restrict__ r, Real* __restrict__ d, Real* __restrict__ x, long long n) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const Real bi = b[i];
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

static unsigned grid_for(long long n) {
  long long b = (n + 255) / 256;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  return (unsigned)b;
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

struct Solver {
  mns_handle* h;
  hipStream_t s;
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

  // dots of w with V_0..V_{K-1} -> host
  int multidot(const double* Vb, int K, const double* wv, double* host) {
    for (int i0 = 0; i0 < K; i0 += 32) {
      const int kk = (K - i0) < 32 ? (K - i0) : 32;
      hipLaunchKernelGGL(k_multidot, dim3(kRedBlocks), dim3(kRedThreads), 0, s, Vb + (size_t)i0 * n, n, kk, wv,
                         parts());
      int rc = reduce(kk);
      if (rc) return rc;
      rc = sync_read(kk, host + i0);
      if (rc) return rc;
    }
    return MNS_OK;
  }

  // host coefficients -> device through the pinned staging half of h_red; the
  // staging area is reused only after a later stream synchronization
  int h2d(const double* host, int K) {
    std::memcpy(h->h_red + 1024, host, K * sizeof(double));
    hipError_t e = hipMemcpyAsync(coefs(), h->h_red + 1024, K * sizeof(double), hipMemcpyHostToDevice, s);
    return e == hipSuccess ? MNS_OK : err(MNS_ERR_HIP, "h2d coefs");
  }

  // w -= V h (h on host), returns ||w||
  int multiaxpy(const double* Vb, int K, const double* hh, double* wv, double* norm) {
    int rc0 = h2d(hh, K);
    if (rc0) return rc0;
    hipLaunchKernelGGL(k_multiaxpy_norm, dim3(kRedBlocks), dim3(kRedThreads), 0, s, Vb, n, K, coefs(), wv, parts());
    int rc = reduce(1);
    if (rc) return rc;
    double v;
    rc = sync_read(1, &v);
    *norm = std::sqrt(v);
    return rc;
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
  int estimate_lambda(int iters, double* lam) {
    // deterministic start vector: 1 on every DoF
    int rc = launch_fill<double>(t64a, 1.0, n, s);
    if (rc) return err(rc, "fill");
    double nrm = std::sqrt((double)n), val = 0;
    hipLaunchKernelGGL(k_scale_copy, dim3(grid_for(n)), dim3(256), 0, s, t64a, 1.0 / nrm, t64a, n);
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
                double range) {
    const double beta = lmax, alpha = lmax / range;
    const double theta = 0.5 * (beta + alpha), delta = 0.5 * (beta - alpha);
    const double sigma = theta / delta;
    double rho = 1.0 / sigma;
    const unsigned g = grid_for(n);
    hipLaunchKernelGGL(k_cheb_init<Real>, dim3(g), dim3(256), 0, s, b, diag, (Real)(1.0 / theta), r, d, x, n);
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

  int precondition(const mns_solve_opts* o, double lmax, const double* v, double* z) {
    const unsigned g = grid_for(n);
    if (o->precond == -1) {
      hipLaunchKernelGGL(k_scale_copy, dim3(g), dim3(256), 0, s, v, 1.0, z, n);
      return MNS_OK;
    }
    if (o->precond == MNS_F64)
      return chebyshev<double>(v, z, r64c, d64c, t64b, h->d_diag64, o->cheb_degree, lmax, o->cheb_range);
    hipLaunchKernelGGL((k_cast<double, float>), dim3(g), dim3(256), 0, s, v, b32, n);
    int rc = chebyshev<float>(b32, x32, r32, d32, t32, h->d_diag32, o->cheb_degree, lmax, o->cheb_range);
    if (rc) return rc;
    hipLaunchKernelGGL((k_cast<float, double>), dim3(g), dim3(256), 0, s, x32, z, n);
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

int ensure_workspace(mns_handle* h, int m) {
  const size_t n = (size_t)h->ndofs;
  hipError_t e;
  if (h->ws_restart < m) {
    if (h->ws64) (void)hipFree(h->ws64);
    h->ws64 = nullptr;
    if ((e = hipMalloc((void**)&h->ws64, (size_t)(2 * m + 9) * n * sizeof(double))) != hipSuccess)
      return set_error(h, MNS_ERR_HIP, std::string("hipMalloc krylov: ") + hipGetErrorString(e));
    h->ws_restart = m;
  }
  if (!h->ws32 && (e = hipMalloc((void**)&h->ws32, 5 * n * sizeof(float))) != hipSuccess)
    return set_error(h, MNS_ERR_HIP, std::string("hipMalloc: ") + hipGetErrorString(e));
  if (!h->d_diag64 && (e = hipMalloc((void**)&h->d_diag64, n * sizeof(double))) != hipSuccess)
    return set_error(h, MNS_ERR_HIP, std::string("hipMalloc: ") + hipGetErrorString(e));
  if (!h->d_diag32 && (e = hipMalloc((void**)&h->d_diag32, n * sizeof(float))) != hipSuccess)
    return set_error(h, MNS_ERR_HIP, std::string("hipMalloc: ") + hipGetErrorString(e));
  if (!h->d_red) {
    if ((e = hipMalloc((void**)&h->d_red, ((size_t)kRedBlocks * 32 + 2048) * sizeof(double))) != hipSuccess)
      return set_error(h, MNS_ERR_HIP, std::string("hipMalloc: ") + hipGetErrorString(e));
    if ((e = hipHostMalloc((void**)&h->h_red, 2048 * sizeof(double), hipHostMallocDefault)) != hipSuccess)
      return set_error(h, MNS_ERR_HIP, std::string("hipHostMalloc: ") + hipGetErrorString(e));
  }
  return MNS_OK;
}

}  // namespace

int mns_solve_impl(mns_handle* h, const double* rhs, double* x, const mns_solve_opts* o, mns_solve_report* rep,
                   hipStream_t s) {
  const auto t0 = std::chrono::steady_clock::now();
  const int m = o->restart;
  int rc = ensure_workspace(h, m);
  if (rc) return rc;
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

  double lmax = 0;
  if (o->precond != -1) {
    if (!h->diag_valid) {
      if ((rc = launch_diagonal<double>(h, h->d_diag64, s))) return rc;
      if ((rc = launch_cast_f64_f32(h->d_diag64, h->d_diag32, (int64_t)n, s))) return set_error(h, rc, "cast");
      h->diag_valid = true;
    }
    if ((rc = S.estimate_lambda(o->eig_iters, &lmax))) return rc;
  }
  rep->lambda_max = lmax;

  // ||b||
  double bn;
  hipLaunchKernelGGL(k_multidot, dim3(kRedBlocks), dim3(kRedThreads), 0, s, rhs, (long long)n, 1, rhs, S.parts());
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
  std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), hcol(m + 1), h2(m + 1), y(m);
  int total = 0, restarts = 0;
  double rnorm = 0;
  bool converged = false;
  while (total < o->maxit) {
    if ((rc = S.true_residual(rhs, x, S.r, &rnorm))) return rc;
    if (rnorm <= target) {
      converged = true;
      break;
    }
    hipLaunchKernelGGL(k_scale_copy, dim3(grid_for(n)), dim3(256), 0, s, S.r, 1.0 / rnorm, S.V, (long long)n);
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = rnorm;
    int j = 0;
    for (; j < m && total < o->maxit; ++j, ++total) {
      double* Vj = S.V + (size_t)j * n;
      double* Zj = S.Z + (size_t)j * n;
      if ((rc = S.precondition(o, lmax, Vj, Zj))) return rc;
      if ((rc = S.jac64(Zj, S.w))) return rc;
      double wn0;
      {
        double v;
        hipLaunchKernelGGL(k_multidot, dim3(kRedBlocks), dim3(kRedThreads), 0, s, S.w, (long long)n, 1, S.w,
                           S.parts());
        if ((rc = S.reduce(1)) || (rc = S.sync_read(1, &v))) return rc;
        wn0 = std::sqrt(v);
      }
      if ((rc = S.multidot(S.V, j + 1, S.w, hcol.data()))) return rc;
      double wn;
      if ((rc = S.multiaxpy(S.V, j + 1, hcol.data(), S.w, &wn))) return rc;
      if (wn < 0.7 * wn0) {  // reorthogonalize once
        if ((rc = S.multidot(S.V, j + 1, S.w, h2.data()))) return rc;
        if ((rc = S.multiaxpy(S.V, j + 1, h2.data(), S.w, &wn))) return rc;
        for (int i = 0; i <= j; ++i) hcol[i] += h2[i];
      }
      hcol[j + 1] = wn;
      if (!std::isfinite(wn)) return set_error(h, MNS_ERR_HIP, "non-finite value in FGMRES");
      // apply earlier rotations, then a new one
      for (int i = 0; i < j; ++i) {
        const double a = cs[i] * hcol[i] + sn[i] * hcol[i + 1];
        const double b = -sn[i] * hcol[i] + cs[i] * hcol[i + 1];
        hcol[i] = a;
        hcol[i + 1] = b;
      }
      const double den = std::hypot(hcol[j], hcol[j + 1]);
      cs[j] = den > 0 ? hcol[j] / den : 1.0;
      sn[j] = den > 0 ? hcol[j + 1] / den : 0.0;
      hcol[j] = den;
      hcol[j + 1] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = hcol[i];
      if (wn > 0)
        hipLaunchKernelGGL(k_scale_copy, dim3(grid_for(n)), dim3(256), 0, s, S.w, 1.0 / wn, S.V + (size_t)(j + 1) * n,
                           (long long)n);
      if (std::fabs(g[j + 1]) <= target || wn == 0) {
        ++j;
        ++total;
        break;
      }
    }
    // y = H^-1 g (upper triangular j x j)
    for (int i = j - 1; i >= 0; --i) {
      double sum = g[i];
      for (int k2 = i + 1; k2 < j; ++k2) sum -= H[(size_t)i * m + k2] * y[k2];
      y[i] = H[(size_t)i * m + i] != 0 ? sum / H[(size_t)i * m + i] : 0.0;
    }
    if ((rc = S.h2d(y.data(), j))) return rc;
    hipLaunchKernelGGL(k_update_x, dim3(grid_for(n)), dim3(256), 0, s, S.Z, (long long)n, j, S.coefs(), x);
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
