// Host-side setup of libmortarns: 1D rules and basis tables, structured mesh
// bookkeeping, element sizes and penalties, the constraint list, and the
// per-angle geometry and mortar tables (all FP64, cast copies for FP32).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "mns_internal.hpp"

namespace mns {

int set_error(mns_handle* h, int code, const std::string& msg) {
  if (h) h->err = msg;
  return code;
}

// Eigenvalues/eigenvectors of a small symmetric matrix by cyclic Jacobi
// rotations (A is overwritten; V receives the eigenvectors as columns).
static void jacobi_eigen(int n, std::vector<double>& A, std::vector<double>& V) {
  V.assign(n * n, 0.0);
  for (int i = 0; i < n; ++i) V[i * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) off += A[p * n + q] * A[p * n + q];
    if (off < 1e-34) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = A[p * n + q];
        if (std::fabs(apq) < 1e-300) continue;
        const double theta = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {  // A <- A J
          const double akp = A[k * n + p], akq = A[k * n + q];
          A[k * n + p] = c * akp - s * akq;
          A[k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {  // A <- J^T A
          const double apk = A[p * n + k], aqk = A[q * n + k];
          A[p * n + k] = c * apk - s * aqk;
          A[q * n + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          const double vkp = V[k * n + p], vkq = V[k * n + q];
          V[k * n + p] = c * vkp - s * vkq;
          V[k * n + q] = s * vkp + c * vkq;
        }
      }
  }
}

// Golub-Welsch: nodes of the m-point Gauss-Jacobi(alpha = beta) rule on
// [-1, 1] as eigenvalues of the symmetric Jacobi matrix; weights (alpha = 0
// only) from the first eigenvector components.
static void golub_welsch(int m, int alpha, std::vector<double>& x, std::vector<double>* w) {
  x.assign(m, 0.0);
  if (w) w->assign(m, 0.0);
  if (m == 0) return;
  std::vector<double> A(m * m, 0.0), V;
  for (int k = 1; k < m; ++k) {
    double b;
    if (alpha == 0) b = k / std::sqrt(4.0 * k * k - 1.0);
    else b = std::sqrt((double)k * (k + 2) / ((2.0 * k + 1) * (2.0 * k + 3)));  // alpha = beta = 1
    A[(k - 1) * m + k] = A[k * m + (k - 1)] = b;
  }
  jacobi_eigen(m, A, V);
  std::vector<int> order(m);
  for (int i = 0; i < m; ++i) order[i] = i;
  std::sort(order.begin(), order.end(), [&](int a, int b) { return A[a * m + a] < A[b * m + b]; });
  for (int i = 0; i < m; ++i) {
    const int j = order[i];
    x[i] = A[j * m + j];
    if (w) (*w)[i] = 2.0 * V[0 * m + j] * V[0 * m + j];
  }
  // symmetric rules: enforce exact symmetry of the nodes
  for (int i = 0; i < m / 2; ++i) {
    const double s = 0.5 * (x[m - 1 - i] - x[i]);
    x[i] = -s;
    x[m - 1 - i] = s;
    if (w) {
      const double ww = 0.5 * ((*w)[i] + (*w)[m - 1 - i]);
      (*w)[i] = (*w)[m - 1 - i] = ww;
    }
  }
  if (m % 2) x[m / 2] = 0.0;
}

void rules_1d(int n, std::vector<double>& gll, std::vector<double>& gx, std::vector<double>& gw) {
  std::vector<double> t, w;
  golub_welsch(n, 0, t, &w);
  gx.resize(n);
  gw.resize(n);
  for (int i = 0; i < n; ++i) {
    gx[i] = 0.5 * (1.0 + t[i]);
    gw[i] = 0.5 * w[i];
  }
  std::vector<double> xi;
  golub_welsch(n - 2, 1, xi, nullptr);  // interior Lobatto nodes: roots of P'_{n-1}
  gll.resize(n);
  gll[0] = 0.0;
  gll[n - 1] = 1.0;
  for (int i = 0; i < n - 2; ++i) gll[i + 1] = 0.5 * (1.0 + xi[i]);
}

// Lagrange basis on `nodes`, value and first two derivatives at t, by
// multiplying in one linear factor at a time (product rule).
void lagrange_1d(const std::vector<double>& nodes, double t, double* L, double* dL, double* d2L) {
  const int n = (int)nodes.size();
  for (int j = 0; j < n; ++j) {
    double p = 1.0, dp = 0.0, d2p = 0.0;
    for (int m = 0; m < n; ++m) {
      if (m == j) continue;
      const double inv = 1.0 / (nodes[j] - nodes[m]);
      const double f = (t - nodes[m]) * inv;
      d2p = d2p * f + 2.0 * dp * inv;
      dp = dp * f + p * inv;
      p = p * f;
    }
    L[j] = p;
    dL[j] = dp;
    d2L[j] = d2p;
  }
}

}  // namespace mns

using namespace mns;

static int hipfail(mns_handle* h, hipError_t e, const char* what) {
  return set_error(h, MNS_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

template <typename T>
static int upload(mns_handle* h, T** dptr, const std::vector<T>& host) {
  if (!*dptr) {
    hipError_t e = hipMalloc((void**)dptr, std::max<size_t>(1, host.size()) * sizeof(T));
    if (e != hipSuccess) return hipfail(h, e, "hipMalloc");
  }
  if (host.empty()) return MNS_OK;
  hipError_t e = hipMemcpy(*dptr, host.data(), host.size() * sizeof(T), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hipfail(h, e, "hipMemcpy");
  return MNS_OK;
}

template <typename T>
static std::vector<float> to_f32(const std::vector<T>& v) {
  std::vector<float> o(v.size());
  for (size_t i = 0; i < v.size(); ++i) o[i] = (float)v[i];
  return o;
}

int mns_build_handle(const mns_mesh_desc* d, hipStream_t stream, mns_handle* h) {
  h->desc = *d;
  h->stream = stream;
  if (d->dim != 2 && d->dim != 3) return set_error(h, MNS_ERR_INVALID_ARG, "dim must be 2 or 3");
  if (d->degree < 2) return set_error(h, MNS_ERR_INVALID_ARG, "degree must be >= 2 (Q1Q1 is unstable at the interface)");
  if ((d->dim == 2 && d->degree > 5) || (d->dim == 3 && d->degree > 4))
    return set_error(h, MNS_ERR_UNSUPPORTED, "degree not compiled (2..5 in 2D, 2..4 in 3D)");
  if (!(d->r_in > 0 && d->r_in < d->r_interface && d->r_interface < d->r_out))
    return set_error(h, MNS_ERR_INVALID_ARG, "radii must satisfy 0 < r_in < r_interface < r_out");
  if (d->n_theta < 3 || d->n_r_rotor < 1 || d->n_r_stator < 1)
    return set_error(h, MNS_ERR_INVALID_ARG, "need n_theta >= 3 and at least one radial cell per domain");
  if (d->n_theta_stator != 0 && d->n_theta_stator < 3)
    return set_error(h, MNS_ERR_INVALID_ARG, "n_theta_stator must be 0 (same as n_theta) or >= 3");
  {
    const int nts = d->n_theta_stator > 0 ? d->n_theta_stator : d->n_theta;
    if (nts > 4 * d->n_theta || d->n_theta > 4 * nts)
      return set_error(h, MNS_ERR_UNSUPPORTED, "interface cell counts more than 4:1 apart");
  }
  if (d->dim == 3 && (d->n_z < 1 || !(d->height > 0)))
    return set_error(h, MNS_ERR_INVALID_ARG, "3D needs n_z >= 1 and height > 0");
  if (!(d->nu > 0) || !std::isfinite(d->nu)) return set_error(h, MNS_ERR_INVALID_ARG, "nu must be > 0");
  if (!(d->penalty_F > 0)) return set_error(h, MNS_ERR_INVALID_ARG, "penalty_F must be > 0");
  if (d->penalty_side_rule != 0 && d->penalty_side_rule != 1)
    return set_error(h, MNS_ERR_INVALID_ARG, "penalty_side_rule must be 0 or 1");
  if (!d->steady && !(d->dt > 0)) return set_error(h, MNS_ERR_INVALID_ARG, "transient needs dt > 0");
  const int k = d->degree;
  h->dim = d->dim;
  h->k = k;
  h->n = k + 1;
  h->nc = d->dim + 1;
  h->nz = d->dim == 3 ? d->n_z : 1;
  h->nth[0] = d->n_theta;
  h->nth[1] = d->n_theta_stator > 0 ? d->n_theta_stator : d->n_theta;
  h->equal_rings = h->nth[0] == h->nth[1];
  for (int dom = 0; dom < 2; ++dom) {
    h->ntd[dom] = k * h->nth[dom];
    h->dthd[dom] = 2.0 * M_PI / h->nth[dom];
  }
  h->ntn = h->ntd[0];
  h->nzn = d->dim == 3 ? k * d->n_z + 1 : 1;
  h->nrn[0] = k * d->n_r_rotor + 1;
  h->nrn[1] = k * d->n_r_stator + 1;
  h->node_off1 = (int64_t)h->ntd[0] * h->nrn[0] * h->nzn;
  h->nnodes = h->node_off1 + (int64_t)h->ntd[1] * h->nrn[1] * h->nzn;
  h->ndofs = h->nnodes * h->nc;
  h->cell_off1 = (int64_t)h->nth[0] * d->n_r_rotor * h->nz;
  h->ncells = h->cell_off1 + (int64_t)h->nth[1] * d->n_r_stator * h->nz;
  if (h->ncells >= (int64_t)1 << 30) return set_error(h, MNS_ERR_UNSUPPORTED, "more than 2^30 cells");
  h->dth = h->dthd[0];
  h->dz = d->dim == 3 ? d->height / d->n_z : 1.0;
  rules_1d(h->n, h->gll, h->gx, h->gw);

  // element size per radial layer: h = 2 sqrt(A/pi) (2D), (6 V/pi)^(1/3) (3D)
  h->hstride = std::max(d->n_r_rotor, d->n_r_stator);
  h->hcell.assign(2 * h->hstride, 0.0);
  const double r0[2] = {d->r_in, d->r_interface};
  const double dr[2] = {(d->r_interface - d->r_in) / d->n_r_rotor, (d->r_out - d->r_interface) / d->n_r_stator};
  const int nr[2] = {d->n_r_rotor, d->n_r_stator};
  for (int dom = 0; dom < 2; ++dom)
    for (int cr = 0; cr < nr[dom]; ++cr) {
      const double ra = r0[dom] + cr * dr[dom], rb = ra + dr[dom];
      const double V = 0.5 * (rb * rb - ra * ra) * h->dthd[dom] * h->dz;
      h->hcell[dom * h->hstride + cr] = d->dim == 2 ? 2.0 * std::sqrt(V / M_PI) : std::cbrt(6.0 * V / M_PI);
    }
  // Hillewaert penalty of the interface cells (Eq. EqPenalty), exact polar measures
  for (int side = 0; side < 2; ++side) {
    const double ra = side == 0 ? d->r_interface - dr[0] : d->r_interface;
    const double rb = side == 0 ? d->r_interface : d->r_interface + dr[1];
    const double other_arc = side == 0 ? ra : rb;
    const double dts = h->dthd[side];
    const double V = 0.5 * (rb * rb - ra * ra) * dts * h->dz;
    const double A_m = d->r_interface * dts * h->dz;
    double A_o = other_arc * dts * h->dz + 2.0 * dr[side] * h->dz;
    if (d->dim == 3) A_o += 2.0 * 0.5 * (rb * rb - ra * ra) * dts;
    h->tau_pen[side] = d->penalty_F * (k + 1.0) * (k + 1.0) * (0.5 * A_o + A_m) / V;
  }
  if (d->penalty_side_rule == 1) h->tau_pen[0] = h->tau_pen[1] = std::max(h->tau_pen[0], h->tau_pen[1]);

  // constraint list: no-slip velocity on r_in (rotor), r_out (stator), z = 0, H;
  // the pinned pressure DoF
  std::vector<int64_t> cons;
  for (int dom = 0; dom < 2; ++dom) {
    const int64_t base = dom ? h->node_off1 : 0;
    for (int iz = 0; iz < h->nzn; ++iz)
      for (int ir = 0; ir < h->nrn[dom]; ++ir) {
        const bool wall = (dom == 0 && ir == 0) || (dom == 1 && ir == h->nrn[1] - 1) ||
                          (d->dim == 3 && (iz == 0 || iz == h->nzn - 1));
        for (int it = 0; it < h->ntd[dom]; ++it) {
          const int64_t node = base + it + (int64_t)h->ntd[dom] * (ir + (int64_t)h->nrn[dom] * iz);
          if (wall)
            for (int c = 0; c < d->dim; ++c) cons.push_back(node * h->nc + c);
          if (dom == 1 && it == 0 && ir == h->nrn[1] - 1 && iz == 0) cons.push_back(node * h->nc + d->dim);
        }
      }
  }
  std::sort(cons.begin(), cons.end());
  h->n_cons = (int64_t)cons.size();
  int rc = upload(h, &h->d_cons, cons);
  if (rc) return rc;
  rc = upload(h, &h->d_hcell64, h->hcell);
  if (rc) return rc;
  rc = upload(h, &h->d_hcell32, to_f32(h->hcell));
  if (rc) return rc;
  // local-result buffers of the volume and mortar kernels (summed by the gather kernel)
  const size_t npt = (size_t)(d->dim == 3 ? h->n * h->n * h->n : h->n * h->n);
  const size_t nE = (size_t)h->ncells * h->nc * npt;
  const size_t nEm = (size_t)(h->nth[0] + h->nth[1]) * h->nz * h->nc * npt;
  hipError_t e;
  if ((e = hipMalloc((void**)&h->d_E64, nE * sizeof(double))) != hipSuccess) return hipfail(h, e, "hipMalloc E");
  if ((e = hipMalloc((void**)&h->d_E32, nE * sizeof(float))) != hipSuccess) return hipfail(h, e, "hipMalloc E");
  if ((e = hipMalloc((void**)&h->d_Em64, nEm * sizeof(double))) != hipSuccess) return hipfail(h, e, "hipMalloc Em");
  if ((e = hipMalloc((void**)&h->d_Em32, nEm * sizeof(float))) != hipSuccess) return hipfail(h, e, "hipMalloc Em");
  // per-angle tables (written by mns_rotate_rotor), the per-point
  // linearization store and the state copy (written by
  // mns_set_linearization): allocated here so that those calls allocate
  // nothing and stay stream-ordered
  const size_t ntrig = (size_t)(h->nth[0] + h->nth[1]) * h->n * 2, nmtrig = (size_t)h->nth[1] * 2 * h->n * 2;
  size_t mtab64 = 0, mtab32 = 0;
  switch (h->n) {
    case 3: mtab64 = sizeof(MortarTab<double, 3>); mtab32 = sizeof(MortarTab<float, 3>); break;
    case 4: mtab64 = sizeof(MortarTab<double, 4>); mtab32 = sizeof(MortarTab<float, 4>); break;
    case 5: mtab64 = sizeof(MortarTab<double, 5>); mtab32 = sizeof(MortarTab<float, 5>); break;
    case 6: mtab64 = sizeof(MortarTab<double, 6>); mtab32 = sizeof(MortarTab<float, 6>); break;
  }
  const int LS = d->dim == 3 ? LinLayout<3>::SIZE : LinLayout<2>::SIZE;
  const size_t nlin = (size_t)h->ncells * npt * LS;
  if ((e = hipMalloc((void**)&h->d_trig64, ntrig * sizeof(double))) != hipSuccess ||
      (e = hipMalloc((void**)&h->d_trig32, ntrig * sizeof(float))) != hipSuccess ||
      (e = hipMalloc((void**)&h->d_mtrig64, nmtrig * sizeof(double))) != hipSuccess ||
      (e = hipMalloc((void**)&h->d_mtrig32, nmtrig * sizeof(float))) != hipSuccess ||
      (e = hipMalloc(&h->d_mtab64, mtab64)) != hipSuccess || (e = hipMalloc(&h->d_mtab32, mtab32)) != hipSuccess)
    return hipfail(h, e, "hipMalloc angle tables");
  if ((e = hipMalloc((void**)&h->d_lin64, nlin * sizeof(double))) != hipSuccess ||
      (e = hipMalloc((void**)&h->d_lin32, nlin * sizeof(float))) != hipSuccess ||
      (e = hipMalloc((void**)&h->d_state, (size_t)h->ndofs * sizeof(double))) != hipSuccess)
    return hipfail(h, e, "hipMalloc linearization store");
  // linearization source C (3D, degrees 2 and 3): tau and tau R per point
  // and an FP32 copy of the state
  if (d->dim == 3 && (d->degree == 2 || d->degree == 3)) {
    const size_t nc4 = (size_t)h->ncells * npt * 4;
    if ((e = hipMalloc((void**)&h->d_linc64, nc4 * sizeof(double))) != hipSuccess ||
        (e = hipMalloc((void**)&h->d_linc32, nc4 * sizeof(float))) != hipSuccess ||
        (e = hipMalloc((void**)&h->d_state32, (size_t)h->ndofs * sizeof(float))) != hipSuccess)
      return hipfail(h, e, "hipMalloc linearization store C");
  }
  // second stream (default priority) and fork/join events of the concurrent
  // launch mode, created here so that no apply call creates them
  if ((e = hipStreamCreateWithFlags(&h->aux, hipStreamNonBlocking)) != hipSuccess ||
      (e = hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming)) != hipSuccess ||
      (e = hipEventCreateWithFlags(&h->ev_join, hipEventDisableTiming)) != hipSuccess)
    return hipfail(h, e, "second stream");
  return MNS_OK;
}

// ---------------------------------------------------------------------------
// Per-angle tables (Sec. 3.1 rotation, Sec. 3.2 mortar segments), built on
// the device by one small kernel so that a rotation is ordered on the
// caller's stream like every other call, synchronizes nothing and can be
// captured into a graph (its arguments are plain values).
// ---------------------------------------------------------------------------
struct RotArgs {
  double theta, phi, dth, R, dz;  // dth, nt: cell angle and ring count of the stator (mortar tables)
  double dthr;                    // cell angle of the rotor ring
  int nt, dim, m;
  int ntr;                        // cells per rotor ring
  double gll[kMaxN], gx[kMaxN], gw[kMaxN];
  double tau_pen[2], inv_dr[2];
};

// Lagrange basis on the N nodes, value and first derivative at t (product
// rule, one linear factor at a time)
template <int N>
__device__ inline void lagrange_dev(const double (&nodes)[kMaxN], double t, double (&L)[N], double (&dL)[N]) {
#pragma unroll
  for (int j = 0; j < N; ++j) {
    double p = 1.0, dp = 0.0;
#pragma unroll
    for (int q = 0; q < N; ++q) {
      if (q == j) continue;
      const double inv = 1.0 / (nodes[j] - nodes[q]);
      const double f = (t - nodes[q]) * inv;
      dp = dp * f + p * inv;
      p = p * f;
    }
    L[j] = p;
    dL[j] = dp;
  }
}

// Work items, in order: (ring cell, Gauss point) cos/sin of the volume
// points, rotor cells first; (stator face, segment, point) cos/sin of the mortar points; (side,
// segment, point) rows of the mortar value/derivative tables; (side) rows of
// the face tables; one item for the weights and scalars.  Segment 0 of stator
// face j spans [j dth, j dth + phi], segment 1 [j dth + phi, (j+1) dth]; the
// theta coordinate of mortar point t on each side:
//   stator: seg 0 xi = t phi/dth,               seg 1 xi = phi/dth + t (1 - phi/dth)
//   rotor:  seg 0 xi = 1 - phi/dth + t phi/dth,  seg 1 xi = t (1 - phi/dth)
template <int N>
__global__ void k_rotate_tables(RotArgs A, double* __restrict__ trig64, float* __restrict__ trig32,
                                double* __restrict__ mtrig64, float* __restrict__ mtrig32,
                                MortarTab<double, N>* __restrict__ M64, MortarTab<float, N>* __restrict__ M32) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int nt = A.nt;
  const long long n_trig = (long long)(A.ntr + nt) * N, n_mtrig = (long long)nt * 2 * N;
  const double len[2] = {A.phi, A.dth - A.phi};
  const double start[2] = {0.0, A.phi};
  if (i < n_trig) {
    const long long row = i / N;
    const int dom = row >= A.ntr;
    const int ct = (int)(dom ? row - A.ntr : row), q = (int)(i % N);
    const double ang = dom == 0 ? A.theta + (ct + A.gx[q]) * A.dthr : (ct + A.gx[q]) * A.dth;
    const double c = cos(ang), sn = sin(ang);
    trig64[2 * i] = c;
    trig64[2 * i + 1] = sn;
    trig32[2 * i] = (float)c;
    trig32[2 * i + 1] = (float)sn;
    return;
  }
  long long j = i - n_trig;
  if (j < n_mtrig) {
    const int face = (int)(j / (2 * N)), sg = (int)((j / N) % 2), q = (int)(j % N);
    const double ang = face * A.dth + start[sg] + A.gx[q] * len[sg];
    const double c = cos(ang), sn = sin(ang);
    mtrig64[2 * j] = c;
    mtrig64[2 * j + 1] = sn;
    mtrig32[2 * j] = (float)c;
    mtrig32[2 * j + 1] = (float)sn;
    return;
  }
  j -= n_mtrig;
  const double f = A.phi / A.dth;
  if (j < 4 * N) {
    const int side = (int)(j / (2 * N)), sg = (int)((j / N) % 2), q = (int)(j % N);
    const double t = A.gx[q];
    const double xi = side == 1 ? (sg == 0 ? t * f : f + t * (1.0 - f)) : (sg == 0 ? 1.0 - f + t * f : t * (1.0 - f));
    double L[N], dL[N];
    lagrange_dev<N>(A.gll, xi, L, dL);
#pragma unroll
    for (int a = 0; a < N; ++a) {
      M64->MV[side][sg][q][a] = L[a];
      M64->MD[side][sg][q][a] = dL[a];
      M32->MV[side][sg][q][a] = (float)L[a];
      M32->MD[side][sg][q][a] = (float)dL[a];
    }
    return;
  }
  j -= 4 * N;
  if (j < 2) {
    const int side = (int)j;
    double L[N], dL[N];
    lagrange_dev<N>(A.gll, side == 0 ? 1.0 : 0.0, L, dL);
#pragma unroll
    for (int b = 0; b < N; ++b) {
      M64->FV[side][b] = L[b];
      M64->FD[side][b] = dL[b];
      M32->FV[side][b] = (float)L[b];
      M32->FD[side][b] = (float)dL[b];
    }
    return;
  }
  if (j != 2) return;
  // Eq. Eq-Jacobian with the segment angle: JxW = w_t R dtheta_seg (w_z dz)
#pragma unroll
  for (int sg = 0; sg < 2; ++sg)
#pragma unroll
    for (int qt = 0; qt < N; ++qt)
#pragma unroll
      for (int qz = 0; qz < N; ++qz) {
        double w = A.gw[qt] * A.R * len[sg];
        if (A.dim == 3) w *= A.gw[qz] * A.dz;
        else if (qz > 0) w = 0.0;
        M64->jxw[sg][qt][qz] = w;
        M32->jxw[sg][qt][qz] = (float)w;
      }
  const double inv_rdth = 1.0 / (A.R * A.dth), inv_dz = A.dim == 3 ? 1.0 / A.dz : 0.0;
  for (int sd = 0; sd < 2; ++sd) {
    M64->tau_pen[sd] = A.tau_pen[sd];
    M32->tau_pen[sd] = (float)A.tau_pen[sd];
    M64->inv_dr[sd] = A.inv_dr[sd];
    M32->inv_dr[sd] = (float)A.inv_dr[sd];
  }
  M64->R = A.R;
  M32->R = (float)A.R;
  M64->inv_rdth = inv_rdth;
  M32->inv_rdth = (float)inv_rdth;
  M64->inv_dz = inv_dz;
  M32->inv_dz = (float)inv_dz;
  const int act0 = A.phi > 0.0 ? 1 : 0;
  M64->seg_active[0] = M32->seg_active[0] = act0;
  M64->seg_active[1] = M32->seg_active[1] = 1;
  M64->m = M32->m = A.m;
}

template <int N>
static int launch_rotate(mns_handle* h, const RotArgs& A, hipStream_t s) {
  const long long items = (long long)(A.ntr + A.nt) * N + (long long)A.nt * 2 * N + 4 * N + 3;
  const unsigned blocks = (unsigned)((items + 255) / 256);
  hipLaunchKernelGGL(k_rotate_tables<N>, dim3(blocks), dim3(256), 0, s, A, h->d_trig64, h->d_trig32, h->d_mtrig64,
                     h->d_mtrig32, (MortarTab<double, N>*)h->d_mtab64, (MortarTab<float, N>*)h->d_mtab32);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? MNS_OK : hipfail(h, e, "rotate kernel");
}

// Rotation x = R(theta) x0 of the rotor (Sec. 3.1) and the mortar tables of
// Sec. 3.2 for that angle, enqueued on stream s.
int mns_rotate_tables(mns_handle* h, double theta, double omega, hipStream_t s) {
  const mns_mesh_desc& d = h->desc;
  const int N = h->n, nt = h->nth[1];
  const double dth = h->dthd[1];
  // theta = m dth + phi with 0 <= phi < dth; snap to alignment within 1e-12 dth
  double mf = std::floor(theta / dth);
  double phi = theta - mf * dth;
  if (phi < 1e-12 * dth) phi = 0.0;
  if (dth - phi < 1e-12 * dth) {
    phi = 0.0;
    mf += 1.0;
  }
  long long m = (long long)std::fmod(mf, (double)nt);
  if (m < 0) m += nt;
  h->theta = theta;
  h->omega = omega;
  h->m = (int)m;
  h->phi = phi;
  RotArgs A{};
  A.theta = theta;
  A.phi = phi;
  A.dth = dth;
  A.dthr = h->dthd[0];
  A.ntr = h->nth[0];
  A.R = d.r_interface;
  A.dz = h->dz;
  A.nt = nt;
  A.dim = d.dim;
  A.m = (int)m;
  for (int q = 0; q < N; ++q) {
    A.gll[q] = h->gll[q];
    A.gx[q] = h->gx[q];
    A.gw[q] = h->gw[q];
  }
  A.tau_pen[0] = h->tau_pen[0];
  A.tau_pen[1] = h->tau_pen[1];
  A.inv_dr[0] = 1.0 / ((d.r_interface - d.r_in) / d.n_r_rotor);
  A.inv_dr[1] = 1.0 / ((d.r_out - d.r_interface) / d.n_r_stator);
  switch (N) {
    case 3: return launch_rotate<3>(h, A, s);
    case 4: return launch_rotate<4>(h, A, s);
    case 5: return launch_rotate<5>(h, A, s);
    case 6: return launch_rotate<6>(h, A, s);
  }
  return set_error(h, MNS_ERR_UNSUPPORTED, "degree");
}
