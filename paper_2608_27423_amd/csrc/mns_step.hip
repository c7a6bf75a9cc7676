// Transient driver: one BDF2 time step of the ALE problem solved by Newton's
// method on the nodal residual (Sec. 2.2 time discretization, Sec. 2.3
// Newton linearization, Sec. 3.1 rotor rotation).  The arithmetic of every
// step is in the operator kernels and the solver; this file adds the
// vector updates and the residual norm.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <vector>

#include "mns_internal.hpp"

namespace mns {

constexpr int kStepBlocks = 1024;

// hist = (-4 u_n + u_nm1) / (2 dt); without u_nm1: -(3 / (2 dt)) u_n
__global__ void k_bdf2_history(const double* __restrict__ un, const double* __restrict__ unm1,
                               double* __restrict__ hist, double inv2dt, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    hist[i] = unm1 ? (unm1[i] - 4.0 * un[i]) * inv2dt : -3.0 * un[i] * inv2dt;
}

// y = a * x (+ y when acc)
__global__ void k_axpy(double a, const double* __restrict__ x, double* __restrict__ y, long long n, int acc) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    y[i] = acc ? y[i] + a * x[i] : a * x[i];
}

// per-block partial sums of x_i^2 (fixed block count and order)
__global__ __launch_bounds__(256) void k_sumsq(const double* __restrict__ x, long long n, double* __restrict__ part) {
  __shared__ double red[256];
  double s = 0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    s += x[i] * x[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

static int step_err(mns_handle* h, hipError_t e, const char* what) {
  return set_error(h, MNS_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

static int norm2(mns_handle* h, const double* x, double* part, hipStream_t s, double* out) {
  const long long n = h->ndofs;
  hipLaunchKernelGGL(k_sumsq, dim3(kStepBlocks), dim3(256), 0, s, x, n, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return step_err(h, e, "norm kernel");
  std::vector<double> host(kStepBlocks);
  if ((e = hipMemcpyAsync(host.data(), part, kStepBlocks * sizeof(double), hipMemcpyDeviceToHost, s)) != hipSuccess ||
      (e = hipStreamSynchronize(s)) != hipSuccess)
    return step_err(h, e, "norm readback");
  double acc = 0;
  for (double v : host) acc += v;
  *out = std::sqrt(acc);
  return MNS_OK;
}

int mns_bdf2_step_impl(mns_handle* h, double theta_next, double omega, const double* un, const double* unm1,
                       const double* force, double* u, const mns_step_opts* o, mns_step_report* rep, hipStream_t s) {
  const auto t0 = std::chrono::steady_clock::now();
  const long long n = h->ndofs;
  hipError_t e;
  if (!h->d_step) {
    if ((e = hipMalloc((void**)&h->d_step, (5 * (size_t)n + kStepBlocks) * sizeof(double))) != hipSuccess)
      return step_err(h, e, "hipMalloc step workspace");
  }
  double* hist = h->d_step;
  double* res = hist + n;
  double* rhs = res + n;
  double* d = rhs + n;
  double* trial = d + n;
  double* part = trial + n;
  const unsigned blocks = kStepBlocks;

  int rc = mns_rotate_rotor(h, theta_next, omega, s);
  if (rc) return rc;
  hipLaunchKernelGGL(k_bdf2_history, dim3(blocks), dim3(256), 0, s, un, unm1, hist, 1.0 / (2.0 * h->desc.dt), n);
  if ((e = hipGetLastError()) != hipSuccess) return step_err(h, e, "history kernel");

  auto done = [&](int status) {
    rep->status = status;
    rep->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return status;
  };
  // Newton with a backtracking line search on ||R||_2: the step u + a d is
  // accepted for the first a in 1, 1/2, 1/4, ... that reduces the norm by the
  // factor (1 - 1e-4 a); after max halvings the smallest step is taken
  constexpr int kMaxHalvings = 8;
  if ((rc = mns_set_linearization(h, u, hist, force, s))) return rc;
  if ((rc = mns_apply_residual(h, u, res, s))) return rc;
  double rn;
  if ((rc = norm2(h, res, part, s, &rn))) return rc;
  const double r0 = rep->residual0 = rep->residual = rn;
  for (int it = 0;; ++it) {
    if (!std::isfinite(rn)) return done(set_error(h, MNS_ERR_NOT_CONVERGED, "residual is not finite"));
    if (rn <= std::fmax(o->newton_atol, o->newton_rtol * r0)) return done(MNS_OK);
    if (it >= o->max_newton) return done(set_error(h, MNS_ERR_NOT_CONVERGED, "Newton iteration limit reached"));
    // J d = -R, zero initial guess
    hipLaunchKernelGGL(k_axpy, dim3(blocks), dim3(256), 0, s, -1.0, res, rhs, n, 0);
    if ((e = hipGetLastError()) != hipSuccess) return step_err(h, e, "vector kernels");
    if ((rc = launch_fill<double>(d, 0.0, n, s))) return set_error(h, rc, "fill");
    mns_solve_report sr{};
    rc = mns_solve(h, rhs, d, &o->linear, &sr, s);
    rep->newton_iterations = it + 1;
    rep->linear_iterations += sr.iterations;
    if (rc == MNS_ERR_NOT_CONVERGED) return done(rc);
    if (rc) return rc;
    double a = 1.0, rt = 0.0;
    for (int ls = 0;; ++ls) {
      hipLaunchKernelGGL(k_axpy, dim3(blocks), dim3(256), 0, s, 1.0, u, trial, n, 0);
      hipLaunchKernelGGL(k_axpy, dim3(blocks), dim3(256), 0, s, a, d, trial, n, 1);
      if ((e = hipGetLastError()) != hipSuccess) return step_err(h, e, "update kernel");
      if ((rc = mns_apply_residual(h, trial, res, s))) return rc;
      if ((rc = norm2(h, res, part, s, &rt))) return rc;
      if ((std::isfinite(rt) && rt <= (1.0 - 1e-4 * a) * rn) || ls == kMaxHalvings) break;
      a *= 0.5;
      ++rep->line_search_halvings;
    }
    hipLaunchKernelGGL(k_axpy, dim3(blocks), dim3(256), 0, s, 1.0, trial, u, n, 0);
    if ((e = hipGetLastError()) != hipSuccess) return step_err(h, e, "update kernel");
    rn = rep->residual = rt;
    if ((rc = mns_set_linearization(h, u, hist, force, s))) return rc;
  }
}

}  // namespace mns
