// Vector kernels over the concatenated vectors of several instances (batched
// FGMRES, batched multigrid levels): blocks of kBChunk entries that never
// straddle two instances, so per-instance scalars are read once per block.
#pragma once

#include <hip/hip_runtime.h>

namespace mns {
namespace {

constexpr int kBT = 256;           // threads per block
constexpr int kBChunk = kBT * 8;   // vector entries per block

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

// Chebyshev scalars of instance i (the recurrence of the single-instance
// polynomial, not contracted) from lambda_max: start 1/theta, step k
// (c1, c2) at cheb[(k count + i) 2 + 0..1]
__device__ inline void cheb_scalars(double lam, double lambda_factor, double range, int deg, int count, int i,
                                    double* inv_theta, double* cheb) {
#pragma clang fp contract(off)
  const double beta = lam * lambda_factor, alpha = beta / range;
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

// out = a + beta c (out may be a)
template <typename Real>
__global__ __launch_bounds__(kBT) void k_baxpy(BSeg S, const Real* a, Real beta, const Real* __restrict__ c, Real* out) {
  int i;
  long long lo, hi;
  bseg_range(S, blockIdx.x, i, lo, hi);
  for (long long q = lo + threadIdx.x; q < hi; q += kBT) out[q] = a[q] + beta * c[q];
}

}  // namespace
}  // namespace mns
