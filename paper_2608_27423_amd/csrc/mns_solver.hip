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

// w -= sum_i h_i V_i ; partial ||w||^2 (coefficients in registers for K <= 32)
__global__ __launch_bounds__(kRedThreads) void k_multiaxpy_norm(const double* __restrict__ V, long long n, int K,
                                                                const double* __restrict__ hcoef,
                                                                double* __restrict__ w, double* __restrict__ part) {
  double acc[1] = {0};
  const long long stride = (long long)gridDim.x * blockDim.x;
  if (K <= kDotK) {
    double hh[kDotK];
#pragma unroll
    for (int i = 0; i < kDotK; ++i) {
      hh[i] = 0.0;
      if (i < K) hh[i] = hcoef[i];
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
      for (int i = 0; i < K; ++i) x -= hcoef[i] * V[(long long)i * n + r];
      w[r] = x;
      acc[0] += x * x;
    }
  }
  block_sum_store<1>(acc, 1, part);
}

// fused Gram-Schmidt pass (K <= 31): w -= sum_i h_i V_i, then partial dots of
// the updated w with V_0 .. V_{K-1} and w . w (entry K), reading V once
__global__ __launch_bounds__(kRedThreads) void k_multiaxpy_dot(const double* __restrict__ V, long long n, int K,
                                                               const double* __restrict__ hcoef,
                                                               double* __restrict__ w, double* __restrict__ part) {
  double hh[kDotK], acc[kDotK];
#pragma unroll
  for (int i = 0; i < kDotK; ++i) {
    hh[i] = 0.0;
    if (i < K) hh[i] = hcoef[i];
    acc[i] = 0;
  }
  const long long stride = (long long)gridDim.x * blockDim.x;
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
  block_sum_store<kDotK>(acc, K + 1, part);
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

struct MG;
int mg_vcycle_in(MG* mg, const mns_solve_opts* o, const double* v, hipStream_t s);
int mg_vcycle_body(MG* mg, const mns_solve_opts* o, hipStream_t s);
int mg_vcycle_out(MG* mg, const mns_solve_opts* o, double* z, hipStream_t s);

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

  // dots of w with V_0..V_{K-1} -> host
  int multidot(const double* Vb, int K, const double* wv, double* host) {
    for (int i0 = 0; i0 < K; i0 += 32) {
      const int kk = (K - i0) < 32 ? (K - i0) : 32;
      hipLaunchKernelGGL(k_multidot, dim3(kRedBlocks), dim3(kRedThreads), 0, s, Vb + (size_t)i0 * n, n, kk, wv,
                         parts(), 0);
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

  // z = M^-1 v in three parts: v is copied (or cast) into a fixed input
  // buffer, the body maps that buffer to a fixed output buffer, which is
  // copied (or cast) to z.  The body's launches depend on neither v nor z, so
  // with use_graph they are captured once per solve and replayed.
  hipGraphExec_t gexec = nullptr;
  int graph_vm64 = 0, graph_vm32 = 0;

  int precond_body(const mns_solve_opts* o, double lmax, hipStream_t bs) {
    Solver B = *this;
    B.s = bs;
    B.vm64 = B.vm32 = 0;
    int rc;
    if (o->precond == MNS_PRECOND_MG || o->precond == MNS_PRECOND_MG64) rc = mg_vcycle_body(mg, o, bs);
    else if (o->precond == MNS_F64)
      rc = B.chebyshev<double>(b64c, d64c + n, r64c, d64c, t64b, h->d_diag64, o->cheb_degree, lmax, o->cheb_range);
    else
      rc = B.chebyshev<float>(b32, x32, r32, d32, t32, h->d_diag32, o->cheb_degree, lmax, o->cheb_range);
    graph_vm64 = B.vm64;
    graph_vm32 = B.vm32;
    return rc;
  }

  int capture_body(const mns_solve_opts* o, double lmax) {
    if (!h->cap && hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking) != hipSuccess)
      return err(MNS_ERR_HIP, "capture stream");
    hipError_t e = hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return err(MNS_ERR_HIP, std::string("begin capture: ") + hipGetErrorString(e));
    const int rc = precond_body(o, lmax, h->cap);
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

  int precondition(const mns_solve_opts* o, double lmax, const double* v, double* z) {
    const unsigned g = grid_for(n);
    if (o->precond == -1) {
      hipLaunchKernelGGL(k_scale_copy, dim3(g), dim3(256), 0, s, v, 1.0, z, n);
      return MNS_OK;
    }
    const bool mgp = o->precond == MNS_PRECOND_MG || o->precond == MNS_PRECOND_MG64;
    int rc;
    if (mgp) {
      if ((rc = mg_vcycle_in(mg, o, v, s))) return rc;
    } else if (o->precond == MNS_F64) {
      hipLaunchKernelGGL(k_scale_copy, dim3(g), dim3(256), 0, s, v, 1.0, b64c, n);
    } else {
      hipLaunchKernelGGL((k_cast<double, float>), dim3(g), dim3(256), 0, s, v, b32, n);
    }
    // graphs need an untimed handle (timed launches record events)
    if (o->use_graph && !h->timing_cap) {
      if (!gexec && (rc = capture_body(o, lmax))) return rc;
      hipError_t e = hipGraphLaunch(gexec, s);
      if (e != hipSuccess) return err(MNS_ERR_HIP, std::string("graph launch: ") + hipGetErrorString(e));
      vm64 += graph_vm64;
      vm32 += graph_vm32;
    } else {
      if ((rc = precond_body(o, lmax, s))) return rc;
      vm64 += graph_vm64;
      vm32 += graph_vm32;
    }
    if (mgp) return mg_vcycle_out(mg, o, z, s);
    if (o->precond == MNS_F64)
      hipLaunchKernelGGL(k_scale_copy, dim3(g), dim3(256), 0, s, (const double*)(d64c + n), 1.0, z, n);
    else
      hipLaunchKernelGGL((k_cast<float, double>), dim3(g), dim3(256), 0, s, x32, z, n);
    return hipGetLastError() == hipSuccess ? MNS_OK : err(MNS_ERR_HIP, "preconditioner copies");
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
    ++h->ws_gen;
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

template <typename Real>
__global__ void k_mg_prolong(TxView X, const Real* __restrict__ coarse, Real* __restrict__ fine, long long nnf,
                             int add) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= nnf) return;
  const int dom = g >= X.off1f;
  const long long l = g - (dom ? X.off1f : 0);
  const int it = (int)(l % X.ntf);
  const long long l2 = l / X.ntf;
  const int nrf = dom ? X.nrf[1] : X.nrf[0];
  const int nrc = dom ? X.nrc[1] : X.nrc[0];
  const int ir = (int)(l2 % nrf), iz = (int)(l2 / nrf);
  const int K1 = X.pw;
  const long long ot = X.pt + (long long)it * K1, orr = (dom ? X.pr[1] : X.pr[0]) + (long long)ir * K1,
                  oz = X.pz + (long long)iz * K1;
  const long long cbase = dom ? X.off1c : 0;
  Real acc[4] = {0, 0, 0, 0};
  for (int a = 0; a < K1; ++a) {
    const double wt = X.w[ot + a];
    if (wt == 0.0) continue;
    for (int b = 0; b < K1; ++b) {
      const double wr = X.w[orr + b];
      if (wr == 0.0) continue;
      for (int c = 0; c < K1; ++c) {
        const double wz = X.w[oz + c];
        if (wz == 0.0) continue;
        const long long node = cbase + X.idx[ot + a] + (long long)X.ntc * (X.idx[orr + b] + (long long)nrc * X.idx[oz + c]);
        const Real ww = (Real)(wt * wr * wz);
        for (int m = 0; m < X.nc; ++m) acc[m] += ww * coarse[node * X.nc + m];
      }
    }
  }
  for (int m = 0; m < X.nc; ++m) fine[g * X.nc + m] = (add ? fine[g * X.nc + m] : Real(0)) + acc[m];
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

template <typename Real>
__global__ void k_mg_restrict_dir(TxView X, RestrictPass P, const Real* __restrict__ in, Real* __restrict__ out,
                                  long long nout) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= nout) return;
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
  for (int m = 0; m < X.nc; ++m) out[g * X.nc + m] = acc[m];
}


// coarse nodal values of a fine field: the fine field evaluated at the
// node counts of the two intermediate grids of the three-pass restriction
static long long restrict_tmp_nodes(const TxView& X) {
  return (long long)X.ntc * X.nzf * (X.nrf[0] + X.nrf[1] + X.nrc[0] + X.nrc[1]);
}

// coarse = P^T fine: theta, then r, then z (tmp holds the intermediate grids)
template <typename Real>
static int mg_restrict(const TxView& X, void* tmp, const Real* fine, Real* coarse, hipStream_t s) {
  Real* t1 = (Real*)tmp;
  const long long n1 = (long long)X.ntc * X.nzf * (X.nrf[0] + X.nrf[1]);
  Real* t2 = t1 + n1 * X.nc;
  const long long n2 = (long long)X.ntc * X.nzf * (X.nrc[0] + X.nrc[1]);
  const long long n3 = (long long)X.ntc * X.nzc * (X.nrc[0] + X.nrc[1]);
  const RestrictPass p1{0, X.ntf, X.nzf, {X.nrf[0], X.nrf[1]}, X.ntc, X.nzf, {X.nrf[0], X.nrf[1]}, X.off1f,
                        (long long)X.ntc * X.nrf[0] * X.nzf};
  const RestrictPass p2{1, X.ntc, X.nzf, {X.nrf[0], X.nrf[1]}, X.ntc, X.nzf, {X.nrc[0], X.nrc[1]}, p1.off1_out,
                        (long long)X.ntc * X.nrc[0] * X.nzf};
  const RestrictPass p3{2, X.ntc, X.nzf, {X.nrc[0], X.nrc[1]}, X.ntc, X.nzc, {X.nrc[0], X.nrc[1]}, p2.off1_out,
                        X.off1c};
  hipLaunchKernelGGL(k_mg_restrict_dir<Real>, dim3((unsigned)((n1 + 255) / 256)), dim3(256), 0, s, X, p1, fine, t1, n1);
  hipLaunchKernelGGL(k_mg_restrict_dir<Real>, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, s, X, p2,
                     (const Real*)t1, t2, n2);
  hipLaunchKernelGGL(k_mg_restrict_dir<Real>, dim3((unsigned)((n3 + 255) / 256)), dim3(256), 0, s, X, p3,
                     (const Real*)t2, coarse, n3);
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
};

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
  MG* mg = new MG();
  mg->max_levels = max_levels;
  h->mg = mg;
  MGLevel L0;
  L0.h = h;
  L0.n = h->ndofs;
  mg->L.push_back(L0);
  mns_mesh_desc d = h->desc;
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
  }
  *out = mg;
  return MNS_OK;
}

// coarse operators at the current angle and state, diagonals and spectra
static int mg_setup(mns_handle* h, MG* mg, const mns_solve_opts* o, hipStream_t s) {
  if (mg->version == h->lin_version && mg->coarse_lin == o->mg_coarse_linearization &&
      mg->fine_lin == o->mg_fine_linearization && mg->eig_iters == o->eig_iters)
    return MNS_OK;
  int rc;
  // level 0: the caller's handle, or a copy of its mesh with the Picard
  // linearization at the same state (the outer FGMRES keeps the caller's)
  if (o->mg_fine_linearization == MNS_LIN_PICARD) {
    if (!mg->fine) {
      mns_handle* hf = new mns_handle();
      if ((rc = mns_build_handle(&h->desc, h->stream, hf))) {
        const std::string msg = hf->err;
        mns_destroy(hf);
        return set_error(h, rc, "multigrid fine copy: " + msg);
      }
      mg->fine = hf;
    }
    mns_handle* hf = mg->fine;
    hf->fused = h->fused;
    hf->quad = h->quad;
    if ((rc = mns_rotate_rotor(hf, h->theta, h->omega))) return set_error(h, rc, "fine copy rotate: " + hf->err);
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
    if ((rc = mns_rotate_rotor(hc, h->theta, h->omega))) return set_error(h, rc, "coarse rotate: " + hc->err);
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
  if (zero) return S.chebyshev<Real>(b, x, v.cr, v.cd, v.ct, v.diag, deg, lmax, range);
  int rc = launch_jacobian<Real>(hl, x, v.ct, s);
  if (rc) return rc;
  hipLaunchKernelGGL(k_mg_axpy<Real>, dim3(g), dim3(256), 0, s, b, Real(-1), (const Real*)v.ct, v.r, Lv.n);
  if ((rc = S.chebyshev<Real>(v.r, v.cx, v.cr, v.cd, v.ct, v.diag, deg, lmax, range))) return rc;
  hipLaunchKernelGGL(k_mg_axpy<Real>, dim3(g), dim3(256), 0, s, (const Real*)x, Real(1), (const Real*)v.cx, x, Lv.n);
  return hipGetLastError() == hipSuccess ? MNS_OK : MNS_ERR_HIP;
}

template <typename Real>
static int mg_cycle(MG* mg, size_t l, const mns_solve_opts* o, hipStream_t s) {
  MGLevel& Lv = mg->L[l];
  mns_handle* hl = Lv.h;
  Solver S = make_solver(hl, s, ws_of(hl, l));
  MGVec<Real> v = mg_vec<Real>(Lv, S);
  int rc;
  if (l + 1 == mg->L.size())
    return mg_smooth<Real>(mg, l, v.b, v.x, true, o->mg_coarse_degree, o->mg_smooth_range, o->cheb_lambda_factor, s);
  if ((rc = mg_smooth<Real>(mg, l, v.b, v.x, true, o->mg_smooth_degree, o->mg_smooth_range, o->cheb_lambda_factor,
                            s)))
    return rc;
  // residual, restricted with constrained rows zero on both levels
  if ((rc = launch_jacobian<Real>(hl, v.x, v.ct, s))) return rc;
  const unsigned g = grid_for(Lv.n);
  hipLaunchKernelGGL(k_mg_axpy<Real>, dim3(g), dim3(256), 0, s, (const Real*)v.b, Real(-1), (const Real*)v.ct, v.r,
                     Lv.n);
  if ((rc = launch_constraints<Real>(hl, v.r, v.r, Real(0), 1, s))) return rc;
  MGLevel& Lc = mg->L[l + 1];
  Solver Sc = make_solver(Lc.h, s, 1);
  MGVec<Real> vc = mg_vec<Real>(Lc, Sc);
  const TxView& X = mg->T[l];
  if ((rc = mg_restrict<Real>(X, Lv.tr, (const Real*)v.r, vc.b, s)))
    return set_error(mg->L[0].h, rc, "multigrid restriction");
  if ((rc = launch_constraints<Real>(Lc.h, vc.b, vc.b, Real(0), 1, s))) return rc;
  if ((rc = mg_cycle<Real>(mg, l + 1, o, s))) return rc;
  // x += P x_c (constrained rows of the correction zero)
  hipLaunchKernelGGL(k_mg_prolong<Real>, dim3((unsigned)((hl->nnodes + 255) / 256)), dim3(256), 0, s, X,
                     (const Real*)vc.x, v.r, (long long)hl->nnodes, 0);
  if ((rc = launch_constraints<Real>(hl, v.r, v.r, Real(0), 1, s))) return rc;
  hipLaunchKernelGGL(k_mg_axpy<Real>, dim3(g), dim3(256), 0, s, (const Real*)v.x, Real(1), (const Real*)v.r, v.x,
                     Lv.n);
  if (hipGetLastError() != hipSuccess) return set_error(mg->L[0].h, MNS_ERR_HIP, "multigrid kernels");
  return mg_smooth<Real>(mg, l, v.b, v.x, false, o->mg_smooth_degree, o->mg_smooth_range, o->cheb_lambda_factor, s);
}

// V-cycle z = B v in three parts (the middle one touches only the levels'
// own vectors, so that it can be captured into a graph): v into level 0's
// right-hand side, the cycle, level 0's iterate into z
int mg_vcycle_in(MG* mg, const mns_solve_opts* o, const double* v, hipStream_t s) {
  MGLevel& L0 = mg->L[0];
  const unsigned g = grid_for(L0.n);
  if (o->precond == MNS_PRECOND_MG64)
    hipLaunchKernelGGL(k_scale_copy, dim3(g), dim3(256), 0, s, v, 1.0, (double*)L0.b, L0.n);
  else
    hipLaunchKernelGGL((k_cast<double, float>), dim3(g), dim3(256), 0, s, v, (float*)L0.b, L0.n);
  return hipGetLastError() == hipSuccess ? MNS_OK : MNS_ERR_HIP;
}

int mg_vcycle_body(MG* mg, const mns_solve_opts* o, hipStream_t s) {
  return o->precond == MNS_PRECOND_MG64 ? mg_cycle<double>(mg, 0, o, s) : mg_cycle<float>(mg, 0, o, s);
}

int mg_vcycle_out(MG* mg, const mns_solve_opts* o, double* z, hipStream_t s) {
  MGLevel& L0 = mg->L[0];
  const unsigned g = grid_for(L0.n);
  if (o->precond == MNS_PRECOND_MG64)
    hipLaunchKernelGGL(k_scale_copy, dim3(g), dim3(256), 0, s, (const double*)L0.b + L0.n, 1.0, z, L0.n);
  else
    hipLaunchKernelGGL((k_cast<float, double>), dim3(g), dim3(256), 0, s, (const float*)L0.b + L0.n, z, L0.n);
  return hipGetLastError() == hipSuccess ? MNS_OK : MNS_ERR_HIP;
}

}  // namespace

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
      if ((rc = S.precondition(o, lmax * o->cheb_lambda_factor, Vj, Zj))) return rc;
      if ((rc = S.jac64(Zj, S.w))) return rc;
      // classical Gram-Schmidt with one reorthogonalization when the norm
      // drops below 0.7 of its value before the projection
      double wn0, wn;
      if (j + 2 <= kDotK) {
        // (1) h = V^T w and w . w in one pass; (2) w -= V h fused with
        // h2 = V^T w and w . w in one pass; (3) only when needed, w -= V h2
        const int K = j + 1;
        double tmp[kDotK + 1];
        hipLaunchKernelGGL(k_multidot, dim3(kRedBlocks), dim3(kRedThreads), 0, s, S.V, (long long)n, K, S.w,
                           S.parts(), 1);
        if ((rc = S.reduce(K + 1)) || (rc = S.sync_read(K + 1, tmp))) return rc;
        for (int i = 0; i < K; ++i) hcol[i] = tmp[i];
        wn0 = std::sqrt(tmp[K]);
        if ((rc = S.h2d(hcol.data(), K))) return rc;
        hipLaunchKernelGGL(k_multiaxpy_dot, dim3(kRedBlocks), dim3(kRedThreads), 0, s, S.V, (long long)n, K,
                           S.coefs(), S.w, S.parts());
        if ((rc = S.reduce(K + 1)) || (rc = S.sync_read(K + 1, tmp))) return rc;
        wn = std::sqrt(tmp[K]);
        if (wn < 0.7 * wn0) {
          for (int i = 0; i < K; ++i) h2[i] = tmp[i];
          if ((rc = S.multiaxpy(S.V, K, h2.data(), S.w, &wn))) return rc;
          for (int i = 0; i < K; ++i) hcol[i] += h2[i];
        }
      } else {
        double v;
        hipLaunchKernelGGL(k_multidot, dim3(kRedBlocks), dim3(kRedThreads), 0, s, S.w, (long long)n, 1, S.w,
                           S.parts(), 0);
        if ((rc = S.reduce(1)) || (rc = S.sync_read(1, &v))) return rc;
        wn0 = std::sqrt(v);
        if ((rc = S.multidot(S.V, j + 1, S.w, hcol.data()))) return rc;
        if ((rc = S.multiaxpy(S.V, j + 1, hcol.data(), S.w, &wn))) return rc;
        if (wn < 0.7 * wn0) {
          if ((rc = S.multidot(S.V, j + 1, S.w, h2.data()))) return rc;
          if ((rc = S.multiaxpy(S.V, j + 1, h2.data(), S.w, &wn))) return rc;
          for (int i = 0; i <= j; ++i) hcol[i] += h2[i];
        }
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

namespace mns {

void mg_free(mns_handle* h) {
  MG* mg = (MG*)h->mg;
  if (!mg) return;
  for (size_t l = 0; l < mg->L.size(); ++l) {
    MGLevel& Lv = mg->L[l];
    if (Lv.b) (void)hipFree(Lv.b);
    if (Lv.inj) (void)hipFree(Lv.inj);
    if (Lv.tr) (void)hipFree(Lv.tr);
    if (l > 0 && Lv.h) mns_destroy(Lv.h);
  }
  if (mg->fine) mns_destroy(mg->fine);
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
                     mg->T[level], x, y, (long long)hf->nnodes, 0);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? MNS_OK : set_error(h, MNS_ERR_HIP, std::string("prolongation: ") + hipGetErrorString(e));
}

}  // namespace mns
