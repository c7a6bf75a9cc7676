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
  h->ntn = k * d->n_theta;
  h->nzn = d->dim == 3 ? k * d->n_z + 1 : 1;
  h->nrn[0] = k * d->n_r_rotor + 1;
  h->nrn[1] = k * d->n_r_stator + 1;
  h->node_off1 = (int64_t)h->ntn * h->nrn[0] * h->nzn;
  h->nnodes = h->node_off1 + (int64_t)h->ntn * h->nrn[1] * h->nzn;
  h->ndofs = h->nnodes * h->nc;
  h->cell_off1 = (int64_t)d->n_theta * d->n_r_rotor * h->nz;
  h->ncells = h->cell_off1 + (int64_t)d->n_theta * d->n_r_stator * h->nz;
  if (h->ncells >= (int64_t)1 << 30) return set_error(h, MNS_ERR_UNSUPPORTED, "more than 2^30 cells");
  h->dth = 2.0 * M_PI / d->n_theta;
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
      const double V = 0.5 * (rb * rb - ra * ra) * h->dth * h->dz;
      h->hcell[dom * h->hstride + cr] = d->dim == 2 ? 2.0 * std::sqrt(V / M_PI) : std::cbrt(6.0 * V / M_PI);
    }
  // Hillewaert penalty of the interface cells (Eq. EqPenalty), exact polar measures
  for (int side = 0; side < 2; ++side) {
    const double ra = side == 0 ? d->r_interface - dr[0] : d->r_interface;
    const double rb = side == 0 ? d->r_interface : d->r_interface + dr[1];
    const double other_arc = side == 0 ? ra : rb;
    const double V = 0.5 * (rb * rb - ra * ra) * h->dth * h->dz;
    const double A_m = d->r_interface * h->dth * h->dz;
    double A_o = other_arc * h->dth * h->dz + 2.0 * dr[side] * h->dz;
    if (d->dim == 3) A_o += 2.0 * 0.5 * (rb * rb - ra * ra) * h->dth;
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
        for (int it = 0; it < h->ntn; ++it) {
          const int64_t node = base + it + (int64_t)h->ntn * (ir + (int64_t)h->nrn[dom] * iz);
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
  const size_t nEm = (size_t)2 * d->n_theta * h->nz * h->nc * npt;
  hipError_t e;
  if ((e = hipMalloc((void**)&h->d_E64, nE * sizeof(double))) != hipSuccess) return hipfail(h, e, "hipMalloc E");
  if ((e = hipMalloc((void**)&h->d_E32, nE * sizeof(float))) != hipSuccess) return hipfail(h, e, "hipMalloc E");
  if ((e = hipMalloc((void**)&h->d_Em64, nEm * sizeof(double))) != hipSuccess) return hipfail(h, e, "hipMalloc Em");
  if ((e = hipMalloc((void**)&h->d_Em32, nEm * sizeof(float))) != hipSuccess) return hipfail(h, e, "hipMalloc Em");
  return MNS_OK;
}

template <typename Real, int N>
static void fill_mortar_tab(const mns_handle* h, MortarTab<Real, N>& M, const double* MV, const double* MD,
                            const double* FV, const double* FD, const double* jxw, const int* active) {
  std::memset(&M, 0, sizeof(M));
  for (int side = 0; side < 2; ++side)
    for (int s = 0; s < 2; ++s)
      for (int q = 0; q < N; ++q)
        for (int a = 0; a < N; ++a) {
          M.MV[side][s][q][a] = (Real)MV[((side * 2 + s) * N + q) * N + a];
          M.MD[side][s][q][a] = (Real)MD[((side * 2 + s) * N + q) * N + a];
        }
  for (int side = 0; side < 2; ++side)
    for (int b = 0; b < N; ++b) {
      M.FV[side][b] = (Real)FV[side * N + b];
      M.FD[side][b] = (Real)FD[side * N + b];
    }
  for (int s = 0; s < 2; ++s)
    for (int qt = 0; qt < N; ++qt)
      for (int qz = 0; qz < N; ++qz) M.jxw[s][qt][qz] = (Real)jxw[(s * N + qt) * N + qz];
  M.tau_pen[0] = (Real)h->tau_pen[0];
  M.tau_pen[1] = (Real)h->tau_pen[1];
  M.R = (Real)h->desc.r_interface;
  const mns_mesh_desc& d = h->desc;
  M.inv_rdth = (Real)(1.0 / (d.r_interface * h->dth));
  M.inv_dr[0] = (Real)(1.0 / ((d.r_interface - d.r_in) / d.n_r_rotor));
  M.inv_dr[1] = (Real)(1.0 / ((d.r_out - d.r_interface) / d.n_r_stator));
  M.inv_dz = d.dim == 3 ? (Real)(1.0 / h->dz) : Real(0);
  M.seg_active[0] = active[0];
  M.seg_active[1] = active[1];
  M.m = h->m;
}

template <int N>
static int upload_mortar(mns_handle* h, const double* MV, const double* MD, const double* FV, const double* FD,
                         const double* jxw, const int* active) {
  MortarTab<double, N> M64;
  MortarTab<float, N> M32;
  fill_mortar_tab<double, N>(h, M64, MV, MD, FV, FD, jxw, active);
  fill_mortar_tab<float, N>(h, M32, MV, MD, FV, FD, jxw, active);
  hipError_t e;
  if (!h->d_mtab64) {
    if ((e = hipMalloc(&h->d_mtab64, sizeof(M64))) != hipSuccess) return hipfail(h, e, "hipMalloc");
    if ((e = hipMalloc(&h->d_mtab32, sizeof(M32))) != hipSuccess) return hipfail(h, e, "hipMalloc");
  }
  if ((e = hipMemcpy(h->d_mtab64, &M64, sizeof(M64), hipMemcpyHostToDevice)) != hipSuccess)
    return hipfail(h, e, "hipMemcpy");
  if ((e = hipMemcpy(h->d_mtab32, &M32, sizeof(M32), hipMemcpyHostToDevice)) != hipSuccess)
    return hipfail(h, e, "hipMemcpy");
  return MNS_OK;
}

// Rotation x = R(theta) x0 of the rotor (Sec. 3.1) and the mortar tables of
// Sec. 3.2 for that angle.
int mns_rotate_tables(mns_handle* h, double theta, double omega) {
  const mns_mesh_desc& d = h->desc;
  const int N = h->n, nt = d.n_theta;
  const double dth = h->dth;
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

  // volume geometry: cos, sin of the physical angle at each Gauss point
  std::vector<double> trig((size_t)2 * nt * N * 2);
  for (int dom = 0; dom < 2; ++dom)
    for (int ct = 0; ct < nt; ++ct)
      for (int q = 0; q < N; ++q) {
        const double ang = (dom == 0 ? theta : 0.0) + (ct + h->gx[q]) * dth;
        trig[(((size_t)dom * nt + ct) * N + q) * 2 + 0] = std::cos(ang);
        trig[(((size_t)dom * nt + ct) * N + q) * 2 + 1] = std::sin(ang);
      }
  // mortar segments of stator face j: [j dth, j dth + phi], [j dth + phi, (j+1) dth]
  const double len[2] = {phi, dth - phi};
  const double start[2] = {0.0, phi};
  const int active[2] = {phi > 0.0 ? 1 : 0, 1};
  std::vector<double> mtrig((size_t)nt * 2 * N * 2);
  for (int j = 0; j < nt; ++j)
    for (int s = 0; s < 2; ++s)
      for (int q = 0; q < N; ++q) {
        const double ang = j * dth + start[s] + h->gx[q] * len[s];
        mtrig[(((size_t)j * 2 + s) * N + q) * 2 + 0] = std::cos(ang);
        mtrig[(((size_t)j * 2 + s) * N + q) * 2 + 1] = std::sin(ang);
      }
  // theta coordinates of the mortar points on each side
  //   stator: seg 0 xi = t phi/dth,          seg 1 xi = phi/dth + t (1 - phi/dth)
  //   rotor:  seg 0 xi = 1 - phi/dth + t phi/dth, seg 1 xi = t (1 - phi/dth)
  const double f = phi / dth;
  std::vector<double> MV(2 * 2 * N * N), MD(2 * 2 * N * N), L(N), dL(N), d2L(N);
  for (int side = 0; side < 2; ++side)
    for (int s = 0; s < 2; ++s)
      for (int q = 0; q < N; ++q) {
        const double t = h->gx[q];
        double xi;
        if (side == 1) xi = s == 0 ? t * f : f + t * (1.0 - f);
        else xi = s == 0 ? 1.0 - f + t * f : t * (1.0 - f);
        lagrange_1d(h->gll, xi, L.data(), dL.data(), d2L.data());
        for (int a = 0; a < N; ++a) {
          MV[((side * 2 + s) * N + q) * N + a] = L[a];
          MD[((side * 2 + s) * N + q) * N + a] = dL[a];
        }
      }
  std::vector<double> FV(2 * N), FD(2 * N);
  for (int side = 0; side < 2; ++side) {
    lagrange_1d(h->gll, side == 0 ? 1.0 : 0.0, L.data(), dL.data(), d2L.data());
    for (int b = 0; b < N; ++b) {
      FV[side * N + b] = L[b];
      FD[side * N + b] = dL[b];
    }
  }
  // Eq. Eq-Jacobian with the segment angle: JxW = w_t R dtheta_seg (w_z dz)
  std::vector<double> jxw(2 * N * N, 0.0);
  for (int s = 0; s < 2; ++s)
    for (int qt = 0; qt < N; ++qt)
      for (int qz = 0; qz < N; ++qz) {
        double w = h->gw[qt] * d.r_interface * len[s];
        if (d.dim == 3) w *= h->gw[qz] * h->dz;
        else if (qz > 0) w = 0.0;
        jxw[(s * N + qt) * N + qz] = w;
      }
  int rc = upload(h, &h->d_trig64, trig);
  if (!rc) rc = upload(h, &h->d_trig32, to_f32(trig));
  if (!rc) rc = upload(h, &h->d_mtrig64, mtrig);
  if (!rc) rc = upload(h, &h->d_mtrig32, to_f32(mtrig));
  if (rc) return rc;
  switch (N) {
    case 3: return upload_mortar<3>(h, MV.data(), MD.data(), FV.data(), FD.data(), jxw.data(), active);
    case 4: return upload_mortar<4>(h, MV.data(), MD.data(), FV.data(), FD.data(), jxw.data(), active);
    case 5: return upload_mortar<5>(h, MV.data(), MD.data(), FV.data(), FD.data(), jxw.data(), active);
    case 6: return upload_mortar<6>(h, MV.data(), MD.data(), FV.data(), FD.data(), jxw.data(), active);
  }
  return set_error(h, MNS_ERR_UNSUPPORTED, "degree");
}
