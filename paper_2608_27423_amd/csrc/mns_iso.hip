// Iso-parametric geometry (the mesh mapping of Sec. 2.1: every cell is the
// Q_k interpolant of its Gauss-Lobatto node positions).  The caller gives the
// node positions once (rotor nodes in the rotor's material frame); the
// library checks them, derives the element sizes and the interface penalty
// (Eq. EqPenalty) from the interpolated cells, and at every rotor angle
// (Sec. 3.1, x = R(theta) x0) rebuilds per Gauss point the inverse Jacobian,
// JxW and the mapping term of the Laplacian that the volume kernels read.
// The mortar integrals stay on the exact interface circle; the inverse
// Jacobians of both sides' interpolated maps at every mortar point are
// rebuilt into a table at every angle as well.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "mns_device.hpp"
#include "mns_internal.hpp"

namespace mns {

// Lagrange basis on the Gauss-Lobatto nodes at N points of [0, 1] (value,
// first and second derivative) and the points' weights
template <int N>
struct IsoTab {
  double V[N][N], D[N][N], DD[N][N];  // [point][node]
  double w[N];
};

// Metric of the interpolated map at every (cell, point) of the table's
// tensor point set: x, J[m][p] = d x_m / d xi_p and the second derivatives
// d^2 x_m / d xi_p d xi_q from the cell's node positions (rotor nodes
// rotated by the angle), then K = J^{-1}, JxW = w |det J|, G = K K^T and the
// mapping term b_p = sum_m K[p][m] sum_pq G_pq d^2 x_m / d xi_p d xi_q.
// flag[0] is set where det J >= 0 (the reference axes (theta, r, z) are
// left-handed, so a cell that keeps the orientation of the polar map has
// det J < 0 everywhere).  geo64 null: the check alone.
template <int DIM, int N>
__global__ __launch_bounds__(256) void k_iso_metric(Geom<double> G, int k, IsoTab<N> P,
                                                    const double* __restrict__ xnode, double crot, double srot,
                                                    double* __restrict__ geo64, float* __restrict__ geo32,
                                                    double* __restrict__ geox, int* __restrict__ flag) {
  using S = Shape<double, DIM, N>;
  using IL = IsoLayout<DIM>;
  constexpr int NZ = S::NZ, NPT = S::NPT;
  const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= G.ncells * NPT) return;
  const int cell = (int)(gid / NPT), pt = (int)(gid % NPT);
  const int q0 = pt % N, q1 = (pt / N) % N, q2 = pt / (N * N);
  const CellId C = decode_cell(G, cell);
  const bool rotor = C.dom == 0;
  double x[3] = {0, 0, 0}, J[3][3] = {}, H[3][6] = {};  // H: 00, 11, 22, 01, 02, 12
  for (int c = 0; c < NZ; ++c) {
    const double z0 = DIM == 3 ? P.V[q2][c] : 1.0, z1 = DIM == 3 ? P.D[q2][c] : 0.0,
                 z2 = DIM == 3 ? P.DD[q2][c] : 0.0;
    for (int b = 0; b < N; ++b) {
      const double r0 = P.V[q1][b], r1 = P.D[q1][b], r2 = P.DD[q1][b];
#pragma unroll
      for (int a = 0; a < N; ++a) {
        const double t0 = P.V[q0][a], t1 = P.D[q0][a], t2 = P.DD[q0][a];
        int it, ir, iz;
        const long long nd = node_of<double, DIM>(G, k, C, a, b, c, it, ir, iz);
        const double X0 = xnode[nd * 3], Y0 = xnode[nd * 3 + 1];
        const double X[3] = {rotor ? crot * X0 - srot * Y0 : X0, rotor ? srot * X0 + crot * Y0 : Y0,
                             xnode[nd * 3 + 2]};
        const double phi = t0 * r0 * z0;
        const double dphi[3] = {t1 * r0 * z0, t0 * r1 * z0, t0 * r0 * z1};
        const double hphi[6] = {t2 * r0 * z0, t0 * r2 * z0, t0 * r0 * z2, t1 * r1 * z0, t1 * r0 * z1, t0 * r1 * z1};
#pragma unroll
        for (int m = 0; m < DIM; ++m) {
          x[m] += phi * X[m];
#pragma unroll
          for (int p = 0; p < DIM; ++p) J[m][p] += dphi[p] * X[m];
#pragma unroll
          for (int i = 0; i < 6; ++i) H[m][i] += hphi[i] * X[m];
        }
      }
    }
  }
  double det, K[3][3] = {};
  if constexpr (DIM == 2) {
    det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    K[0][0] = J[1][1] / det;
    K[0][1] = -J[0][1] / det;
    K[1][0] = -J[1][0] / det;
    K[1][1] = J[0][0] / det;
  } else {
    const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
    K[0][0] = c00 / det;
    K[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
    K[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
    K[1][0] = c01 / det;
    K[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
    K[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
    K[2][0] = c02 / det;
    K[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
    K[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
  }
  if (!(det < 0.0)) flag[0] = 1;
  if (!geo64) return;
  double Gm[3][3];
#pragma unroll
  for (int p = 0; p < DIM; ++p)
#pragma unroll
    for (int q = 0; q < DIM; ++q) {
      double t = 0;
#pragma unroll
      for (int m = 0; m < DIM; ++m) t += K[p][m] * K[q][m];
      Gm[p][q] = t;
    }
  double cm[3];
#pragma unroll
  for (int m = 0; m < DIM; ++m) {
    double t = Gm[0][0] * H[m][0] + Gm[1][1] * H[m][1] + 2.0 * Gm[0][1] * H[m][3];
    if constexpr (DIM == 3) t += Gm[2][2] * H[m][2] + 2.0 * (Gm[0][2] * H[m][4] + Gm[1][2] * H[m][5]);
    cm[m] = t;
  }
  double w = P.w[q0] * P.w[q1];
  if constexpr (DIM == 3) w *= P.w[q2];
  double out[IL::SIZE];
#pragma unroll
  for (int p = 0; p < DIM; ++p)
#pragma unroll
    for (int m = 0; m < DIM; ++m) out[IL::K + p * DIM + m] = K[p][m];
  out[IL::JXW] = w * fabs(det);
#pragma unroll
  for (int p = 0; p < DIM; ++p) {
    double t = 0;
#pragma unroll
    for (int m = 0; m < DIM; ++m) t += K[p][m] * cm[m];
    out[IL::B + p] = t;
  }
  double* g64 = geo64 + gid * IL::SIZE;
  float* g32 = geo32 + gid * IL::SIZE;
#pragma unroll
  for (int j = 0; j < IL::SIZE; ++j) {
    g64[j] = out[j];
    g32[j] = (float)out[j];
  }
#pragma unroll
  for (int m = 0; m < 3; ++m) geox[gid * 3 + m] = m < DIM ? x[m] : 0.0;
}

// element size of every cell from its volume (sum of JxW): h = 2 sqrt(A/pi)
// in 2D, (6 V / pi)^(1/3) in 3D, the rule of the polar cells
template <int DIM>
__global__ void k_iso_h(const double* __restrict__ geo64, long long ncells, int npt, double* __restrict__ hcell) {
  using IL = IsoLayout<DIM>;
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncells) return;
  double V = 0;
  for (int p = 0; p < npt; ++p) V += geo64[(c * npt + p) * IL::SIZE + IL::JXW];
  hcell[c] = DIM == 2 ? 2.0 * sqrt(V / M_PI) : cbrt(6.0 * V / M_PI);
}

namespace {

Geom<double> index_geom(const mns_handle* h) {
  Geom<double> G{};
  G.ncells = h->ncells;
  G.cell_off1 = h->cell_off1;
  G.node_off1 = h->node_off1;
  G.ndofs = h->ndofs;
  for (int d = 0; d < 2; ++d) {
    G.nth[d] = h->nth[d];
    G.ntd[d] = h->ntd[d];
    G.nrn[d] = h->nrn[d];
  }
  G.nr[0] = h->desc.n_r_rotor;
  G.nr[1] = h->desc.n_r_stator;
  G.nz = h->nz;
  G.nzn = h->nzn;
  return G;
}

template <int N>
IsoTab<N> iso_tab(const mns_handle* h, const std::vector<double>& pts, const std::vector<double>& w) {
  IsoTab<N> P{};
  std::vector<double> L(N), dL(N), d2L(N);
  for (int q = 0; q < N; ++q) {
    lagrange_1d(h->gll, pts[q], L.data(), dL.data(), d2L.data());
    for (int a = 0; a < N; ++a) {
      P.V[q][a] = L[a];
      P.D[q][a] = dL[a];
      P.DD[q][a] = d2L[a];
    }
    P.w[q] = w[q];
  }
  return P;
}

// global node of local node (a, b, c) of cell (dom, ct, cr, cz)
int64_t host_node(const mns_handle* h, int dom, int ct, int cr, int cz, int a, int b, int c) {
  const int k = h->k, ntn = h->ntd[dom];
  int it = k * ct + a;
  if (it >= ntn) it -= ntn;
  const int64_t ir = (int64_t)k * cr + b, iz = h->dim == 3 ? (int64_t)k * cz + c : 0;
  return (dom ? h->node_off1 : 0) + it + (int64_t)ntn * (ir + (int64_t)h->nrn[dom] * iz);
}

// J[m][p] of the interpolated map of a cell at reference point xi
void host_jacobian(const mns_handle* h, const double* xyz, int dom, int ct, int cr, int cz, const double xi[3],
                   double J[3][3]) {
  const int n = h->n, d = h->dim;
  std::vector<double> L[3], dL[3], d2L[3];
  for (int e = 0; e < 3; ++e) {
    L[e].assign(n, 1.0);
    dL[e].assign(n, 0.0);
    d2L[e].assign(n, 0.0);
    if (e < d) lagrange_1d(h->gll, xi[e], L[e].data(), dL[e].data(), d2L[e].data());
  }
  for (int m = 0; m < 3; ++m)
    for (int p = 0; p < 3; ++p) J[m][p] = 0;
  const int nzn = d == 3 ? n : 1;
  for (int c = 0; c < nzn; ++c)
    for (int b = 0; b < n; ++b)
      for (int a = 0; a < n; ++a) {
        const int64_t nd = host_node(h, dom, ct, cr, cz, a, b, c);
        const int idx[3] = {a, b, c};
        for (int p = 0; p < d; ++p) {
          double v = 1.0;
          for (int e = 0; e < d; ++e) v *= (e == p) ? dL[e][idx[e]] : L[e][idx[e]];
          for (int m = 0; m < d; ++m) J[m][p] += v * xyz[nd * 3 + m];
        }
      }
}

// volume and the area of the face xi_dir = val of a cell, by the Gauss rule
// on the interpolated map
double host_volume(const mns_handle* h, const double* xyz, int dom, int ct, int cr, int cz) {
  const int n = h->n, d = h->dim;
  double V = 0;
  for (int q2 = 0; q2 < (d == 3 ? n : 1); ++q2)
    for (int q1 = 0; q1 < n; ++q1)
      for (int q0 = 0; q0 < n; ++q0) {
        const double xi[3] = {h->gx[q0], h->gx[q1], d == 3 ? h->gx[q2] : 0.0};
        double J[3][3];
        host_jacobian(h, xyz, dom, ct, cr, cz, xi, J);
        const double det = d == 2 ? J[0][0] * J[1][1] - J[0][1] * J[1][0]
                                  : J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                                        J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                                        J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
        V += h->gw[q0] * h->gw[q1] * (d == 3 ? h->gw[q2] : 1.0) * std::fabs(det);
      }
  return V;
}

double host_face(const mns_handle* h, const double* xyz, int dom, int ct, int cr, int cz, int dir, double val) {
  const int n = h->n, d = h->dim;
  int other[2] = {0, 0}, no = 0;
  for (int e = 0; e < d; ++e)
    if (e != dir) other[no++] = e;
  double A = 0;
  for (int q1 = 0; q1 < (d == 3 ? n : 1); ++q1)
    for (int q0 = 0; q0 < n; ++q0) {
      double xi[3] = {0, 0, 0};
      xi[dir] = val;
      xi[other[0]] = h->gx[q0];
      double w = h->gw[q0];
      if (d == 3) {
        xi[other[1]] = h->gx[q1];
        w *= h->gw[q1];
      }
      double J[3][3];
      host_jacobian(h, xyz, dom, ct, cr, cz, xi, J);
      const double t0[3] = {J[0][other[0]], J[1][other[0]], J[2][other[0]]};
      if (d == 2) {
        A += w * std::sqrt(t0[0] * t0[0] + t0[1] * t0[1]);
      } else {
        const double t1[3] = {J[0][other[1]], J[1][other[1]], J[2][other[1]]};
        const double cx = t0[1] * t1[2] - t0[2] * t1[1], cy = t0[2] * t1[0] - t0[0] * t1[2],
                     cz2 = t0[0] * t1[1] - t0[1] * t1[0];
        A += w * std::sqrt(cx * cx + cy * cy + cz2 * cz2);
      }
    }
  return A;
}

template <int DIM, int N>
int launch_metric(mns_handle* h, const IsoTab<N>& P, double theta, bool tables, hipStream_t s) {
  const long long total = (long long)h->ncells * Shape<double, DIM, N>::NPT;
  hipLaunchKernelGGL((k_iso_metric<DIM, N>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, index_geom(h),
                     h->k, P, (const double*)h->d_xnode, std::cos(theta), std::sin(theta),
                     tables ? h->d_geo64 : nullptr, h->d_geo32, h->d_geox, h->d_iso_flag);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? MNS_OK : set_error(h, MNS_ERR_HIP, std::string("iso metric kernel: ") + hipGetErrorString(e));
}

// the metric at the Gauss points (tables) or the orientation check alone at
// the Gauss-Lobatto points
int metric(mns_handle* h, double theta, bool gauss, hipStream_t s) {
  const std::vector<double> ones(h->n, 1.0);
#define MNS_ISO_CASE(D, NN)                                                                        \
  if (h->dim == D && h->n == NN)                                                                   \
    return launch_metric<D, NN>(h, gauss ? iso_tab<NN>(h, h->gx, h->gw) : iso_tab<NN>(h, h->gll, ones), theta, \
                                gauss, s);
  MNS_ISO_CASE(2, 3) MNS_ISO_CASE(2, 4) MNS_ISO_CASE(2, 5) MNS_ISO_CASE(2, 6)
  MNS_ISO_CASE(3, 3) MNS_ISO_CASE(3, 4) MNS_ISO_CASE(3, 5)
#undef MNS_ISO_CASE
  return set_error(h, MNS_ERR_UNSUPPORTED, "degree not compiled");
}

int hipfail(mns_handle* h, hipError_t e, const char* what) {
  return set_error(h, MNS_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace

int iso_set_nodes(mns_handle* h, const double* xyz, int64_t n_nodes, hipStream_t s) {
  const mns_mesh_desc& d = h->desc;
  if (!h->iso) {
    h->tau_pen_polar[0] = h->tau_pen[0];
    h->tau_pen_polar[1] = h->tau_pen[1];
  }
  if (!xyz) {
    h->iso = false;
    h->tau_pen[0] = h->tau_pen_polar[0];
    h->tau_pen[1] = h->tau_pen_polar[1];
    return MNS_OK;
  }
  if (n_nodes != h->nnodes)
    return set_error(h, MNS_ERR_INVALID_ARG,
                     "n_nodes must be the mesh's node count " + std::to_string((long long)h->nnodes));
  for (int64_t i = 0; i < 3 * n_nodes; ++i)
    if (!std::isfinite(xyz[i])) return set_error(h, MNS_ERR_INVALID_ARG, "node positions must be finite");
  // the mortar quadrature lives on the exact interface circle with the polar
  // parameterization of the faces: interface nodes must sit at their polar
  // positions
  const double tol = 1e-10 * std::max(d.r_interface, d.dim == 3 ? d.height : 0.0);
  for (int dom = 0; dom < 2; ++dom) {
    const int ir = dom == 0 ? h->nrn[0] - 1 : 0;
    for (int iz = 0; iz < h->nzn; ++iz)
      for (int it = 0; it < h->ntd[dom]; ++it) {
        const int64_t nd = (dom ? h->node_off1 : 0) + it + (int64_t)h->ntd[dom] * (ir + (int64_t)h->nrn[dom] * iz);
        const double th = (it / h->k + h->gll[it % h->k]) * h->dthd[dom];
        const double z = d.dim == 3 ? (iz / h->k + h->gll[iz % h->k]) * h->dz : 0.0;
        const double ex = d.r_interface * std::cos(th), ey = d.r_interface * std::sin(th);
        if (std::fabs(xyz[nd * 3] - ex) > tol || std::fabs(xyz[nd * 3 + 1] - ey) > tol ||
            (d.dim == 3 && std::fabs(xyz[nd * 3 + 2] - z) > tol))
          return set_error(h, MNS_ERR_INVALID_ARG,
                           "interface node " + std::to_string((long long)nd) +
                               " is not at its polar position on the interface circle");
      }
  }
  // penalty of the interface cells (Eq. EqPenalty) from the interpolated
  // cell at ring index 0 and layer 0 of each side
  double tau[2];
  for (int side = 0; side < 2; ++side) {
    const int cr = side == 0 ? d.n_r_rotor - 1 : 0;
    const double V = host_volume(h, xyz, side, 0, cr, 0);
    const double Am = host_face(h, xyz, side, 0, cr, 0, 1, side == 0 ? 1.0 : 0.0);
    double Ao = host_face(h, xyz, side, 0, cr, 0, 1, side == 0 ? 0.0 : 1.0) + host_face(h, xyz, side, 0, cr, 0, 0, 0.0) +
                host_face(h, xyz, side, 0, cr, 0, 0, 1.0);
    if (d.dim == 3) Ao += host_face(h, xyz, side, 0, cr, 0, 2, 0.0) + host_face(h, xyz, side, 0, cr, 0, 2, 1.0);
    if (!(V > 0)) return set_error(h, MNS_ERR_INVALID_ARG, "degenerate interface cell");
    tau[side] = d.penalty_F * (h->k + 1.0) * (h->k + 1.0) * (0.5 * Ao + Am) / V;
  }
  if (d.penalty_side_rule == 1) tau[0] = tau[1] = std::max(tau[0], tau[1]);
  // device tables (allocated by the first call, kept)
  const size_t npt = (size_t)(d.dim == 3 ? h->n * h->n * h->n : h->n * h->n);
  const size_t ngeo = (size_t)h->ncells * npt * (d.dim == 3 ? IsoLayout<3>::SIZE : IsoLayout<2>::SIZE);
  hipError_t e;
  if (!h->d_xnode) {
    if ((e = hipMalloc((void**)&h->d_xnode, (size_t)h->nnodes * 3 * sizeof(double))) != hipSuccess ||
        (e = hipMalloc((void**)&h->d_geo64, ngeo * sizeof(double))) != hipSuccess ||
        (e = hipMalloc((void**)&h->d_geo32, ngeo * sizeof(float))) != hipSuccess ||
        (e = hipMalloc((void**)&h->d_geox, (size_t)h->ncells * npt * 3 * sizeof(double))) != hipSuccess ||
        (e = hipMalloc((void**)&h->d_hiso, (size_t)h->ncells * sizeof(double))) != hipSuccess ||
        (e = hipMalloc((void**)&h->d_iso_flag, sizeof(int))) != hipSuccess)
      return hipfail(h, e, "hipMalloc iso-parametric tables");
    // mortar point geometry: face sides x segment slots x points
    h->mgeo_pieces = iso_mortar_pieces(h);
    const size_t nmg = (size_t)(h->nth[0] + h->nth[1]) * h->nz * h->mgeo_pieces * (d.dim == 3 ? h->n * h->n : h->n) *
                       (d.dim == 3 ? IsoMortarLayout<3>::SIZE : IsoMortarLayout<2>::SIZE);
    if ((e = hipMalloc((void**)&h->d_mgeo64, nmg * sizeof(double))) != hipSuccess ||
        (e = hipMalloc((void**)&h->d_mgeo32, nmg * sizeof(float))) != hipSuccess)
      return hipfail(h, e, "hipMalloc iso-parametric mortar tables");
  }
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return hipfail(h, e, "synchronize");
  const int zero = 0;
  if ((e = hipMemcpy(h->d_xnode, xyz, (size_t)n_nodes * 3 * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(h->d_iso_flag, &zero, sizeof(int), hipMemcpyHostToDevice)) != hipSuccess)
    return hipfail(h, e, "copy node positions");
  // orientation at every Gauss-Lobatto point (faces and corners included),
  // then the metric at the Gauss points (angle 0) and the element sizes
  int rc;
  if ((rc = metric(h, 0.0, false, s))) return rc;
  if ((rc = metric(h, 0.0, true, s))) return rc;
  const long long nc = h->ncells;
  if (d.dim == 3)
    hipLaunchKernelGGL(k_iso_h<3>, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, s, h->d_geo64, nc, (int)npt,
                       h->d_hiso);
  else
    hipLaunchKernelGGL(k_iso_h<2>, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, s, h->d_geo64, nc, (int)npt,
                       h->d_hiso);
  if ((e = hipGetLastError()) != hipSuccess) return hipfail(h, e, "element size kernel");
  int folded = 0;
  if ((e = hipStreamSynchronize(s)) != hipSuccess ||
      (e = hipMemcpy(&folded, h->d_iso_flag, sizeof(int), hipMemcpyDeviceToHost)) != hipSuccess)
    return hipfail(h, e, "read orientation flag");
  if (folded) {
    h->iso = false;
    h->tau_pen[0] = h->tau_pen_polar[0];
    h->tau_pen[1] = h->tau_pen_polar[1];
    return set_error(h, MNS_ERR_INVALID_ARG,
                     "node positions fold a cell: det J of the interpolated map is zero or of the wrong sign");
  }
  h->tau_pen[0] = tau[0];
  h->tau_pen[1] = tau[1];
  h->iso = true;
  return MNS_OK;
}

int iso_rotate(mns_handle* h, double theta, hipStream_t s) {
  if (!h->iso) return MNS_OK;
  const int rc = metric(h, theta, true, s);
  return rc ? rc : launch_iso_mortar_geo(h, s);
}

}  // namespace mns
