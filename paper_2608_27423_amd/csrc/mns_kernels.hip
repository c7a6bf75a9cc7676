// Volume, mortar, diagonal and constraint kernels of the stabilized ALE
// Navier-Stokes Jacobian (gfx950).
//
// Work decomposition of the volume kernels: one 64-lane wavefront per block;
// each cell is handled by N*N lanes (lane t owns the node/point line at
// (i_theta, i_r) = (t % N, t / N) along z).  The z contraction of the
// sum-factorized evaluation runs in registers, the r and theta contractions
// go through LDS.  2D is the same code with a line of length one.
//
// Scatter without atomics: every cell (and mortar cell side) stores its local
// result; k_gather sums the contributions of each node in a fixed order and
// applies the constraint rows, so the product is bitwise reproducible.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>
#include <mutex>
#include <string>
#include <type_traits>

#include <hip/hip_ext.h>

#include "mns_device.hpp"
#include "mns_internal.hpp"

namespace mns {

// constraint predicates, written with bitwise operators so that they
// compile to selects rather than branches
template <typename Real, int DIM>
__device__ inline bool vel_fixed(const Geom<Real>& G, int dom, int ir, int iz) {
  const bool wall_r = ((dom == 0) & (ir == 0)) | ((dom == 1) & (ir == G.nrn[1] - 1));
  const bool wall_z = (DIM == 3) & ((iz == 0) | (iz == G.nzn - 1));
  return wall_r | wall_z;
}

template <typename Real>
__device__ inline bool p_fixed(const Geom<Real>& G, int dom, int it, int ir, int iz) {
  return (dom == 1) & (it == 0) & (ir == G.nrn[1] - 1) & (iz == 0);
}

template <typename T>
__device__ inline void atomic_add(T* p, T v) {
  unsafeAtomicAdd(p, v);
}

// ---------------------------------------------------------------------------
// Evaluation: nodal line values -> reference values and derivatives at the
// lane's points (i_theta = tqi, i_r = tqj, all z points).
// ---------------------------------------------------------------------------

// reference derivatives of one component at one point
template <typename Real, int DIM>
struct RefVal {
  Real v;
  Real d[DIM];   // d/dxi_theta, d/dxi_r [, d/dxi_z]
  Real dd[DIM];  // second derivatives along the same directions
};

// Stage 1 of the evaluation (z in registers) and write to LDS; u[comp][c] is
// the lane's nodal line.  Velocity components use slots comp*NYV + {0: V,
// 1: D, 2: DD}; the pressure slots DIM*NYV + {0: V, 1: D}.  In 2D the line has
// one node and only the value slot is written.
template <typename Real, int DIM, int N, int NCOMP_V, bool PRES>
__device__ inline void eval_stage_z(const Tab1D<Real, N>& T, const Real (*u)[Shape<Real, DIM, N>::NZ], Real* L,
                                    int ta, int tb, bool active) {
  using S = Shape<Real, DIM, N>;
  constexpr int NZ = S::NZ;
  if (!active) return;
#pragma unroll
  for (int m = 0; m < NCOMP_V + (PRES ? 1 : 0); ++m) {
    const bool vel = m < NCOMP_V;
    const int base = vel ? m * S::NYV : NCOMP_V * S::NYV;
    if constexpr (DIM == 3) {
#pragma unroll
      for (int q = 0; q < NZ; ++q) {
        Real sv = 0, sd = 0, sdd = 0;
#pragma unroll
        for (int c = 0; c < NZ; ++c) {
          sv += T.V[q][c] * u[m][c];
          sd += T.D[q][c] * u[m][c];
          if (vel) sdd += T.DD[q][c] * u[m][c];
        }
        const int idx = q * S::PLANE + tb * N + ta;
        L[((base + 0) * S::NPT + idx) * S::ES] = sv;
        L[((base + 1) * S::NPT + idx) * S::ES] = sd;
        if (vel) L[((base + 2) * S::NPT + idx) * S::ES] = sdd;
      }
    } else {
      L[(base * S::NPT + tb * N + ta) * S::ES] = u[m][0];
    }
  }
}

// Stage 2 (r through LDS).  Lane (ta, tqj) reads the column (b = 0..N-1) of
// its theta node and writes back, after a barrier, the r-contracted arrays:
// velocity {VV, DV, DDV, VD, VDD} (3D) or {V, D, DD} (2D); pressure {VV, DV, VD}
// (3D) or {V, D} (2D).  First letter: r operator, second: z operator.
template <typename Real, int DIM, int N, int NCOMP_V, bool PRES>
__device__ inline void eval_stage_r(const Tab1D<Real, N>& T, Real* L, int ta, int tqj, bool active) {
  using S = Shape<Real, DIM, N>;
  constexpr int NZ = S::NZ;
  constexpr int NF = NCOMP_V + (PRES ? 1 : 0);
  Real out[NF][S::NYV][NZ];
  if (active) {
#pragma unroll
    for (int m = 0; m < NF; ++m) {
      const bool vel = m < NCOMP_V;
      const int base = vel ? m * S::NYV : NCOMP_V * S::NYV;
#pragma unroll
      for (int q = 0; q < NZ; ++q) {
        Real vv = 0, dv = 0, ddv = 0, vd = 0, vdd = 0;
#pragma unroll
        for (int b = 0; b < N; ++b) {
          const int idx = q * S::PLANE + b * N + ta;
          const Real zv = L[((base + 0) * S::NPT + idx) * S::ES];
          vv += T.V[tqj][b] * zv;
          dv += T.D[tqj][b] * zv;
          if (vel) ddv += T.DD[tqj][b] * zv;
          if constexpr (DIM == 3) {
            const Real zd = L[((base + 1) * S::NPT + idx) * S::ES];
            vd += T.V[tqj][b] * zd;
            if (vel) vdd += T.V[tqj][b] * L[((base + 2) * S::NPT + idx) * S::ES];
          }
        }
        out[m][0][q] = vv;
        out[m][1][q] = dv;
        if constexpr (DIM == 3) {
          if (vel) {
            out[m][2][q] = ddv;
            out[m][3][q] = vd;
            out[m][4][q] = vdd;
          } else {
            out[m][2][q] = vd;
          }
        } else {
          if (vel) out[m][2][q] = ddv;
        }
      }
    }
  }
  __syncthreads();
  if (active) {
#pragma unroll
    for (int m = 0; m < NF; ++m) {
      const bool vel = m < NCOMP_V;
      const int base = vel ? m * S::NYV : NCOMP_V * S::NYV;
      const int nout = vel ? S::NYV : S::NYP;
#pragma unroll
      for (int j = 0; j < S::NYV; ++j) {
        if (j >= nout) break;
#pragma unroll
        for (int q = 0; q < NZ; ++q) L[((base + j) * S::NPT + q * S::PLANE + tqj * N + ta) * S::ES] = out[m][j][q];
      }
    }
  }
  __syncthreads();
}

// Stage 3 (theta through LDS) for one z point q: lane (tqi, tqj).
template <typename Real, int DIM, int N>
__device__ inline void eval_stage_t_vel(const Tab1D<Real, N>& T, const Real* L, int base, int tqi, int tqj, int q,
                                        RefVal<Real, DIM>& r) {
  using S = Shape<Real, DIM, N>;
  Real v = 0, dt = 0, ddt = 0, dr = 0, ddr = 0, dz = 0, ddz = 0;
#pragma unroll
  for (int a = 0; a < N; ++a) {
    const int idx = q * S::PLANE + tqj * N + a;
    const Real yvv = L[((base + 0) * S::NPT + idx) * S::ES];
    v += T.V[tqi][a] * yvv;
    dt += T.D[tqi][a] * yvv;
    ddt += T.DD[tqi][a] * yvv;
    dr += T.V[tqi][a] * L[((base + 1) * S::NPT + idx) * S::ES];
    ddr += T.V[tqi][a] * L[((base + 2) * S::NPT + idx) * S::ES];
    if constexpr (DIM == 3) {
      dz += T.V[tqi][a] * L[((base + 3) * S::NPT + idx) * S::ES];
      ddz += T.V[tqi][a] * L[((base + 4) * S::NPT + idx) * S::ES];
    }
  }
  r.v = v;
  r.d[0] = dt;
  r.d[1] = dr;
  r.dd[0] = ddt;
  r.dd[1] = ddr;
  if constexpr (DIM == 3) {
    r.d[2] = dz;
    r.dd[2] = ddz;
  }
}

template <typename Real, int DIM, int N>
__device__ inline void eval_stage_t_pres(const Tab1D<Real, N>& T, const Real* L, int base, int tqi, int tqj, int q,
                                         RefVal<Real, DIM>& r) {
  using S = Shape<Real, DIM, N>;
  Real v = 0, dt = 0, dr = 0, dz = 0;
#pragma unroll
  for (int a = 0; a < N; ++a) {
    const int idx = q * S::PLANE + tqj * N + a;
    const Real yvv = L[((base + 0) * S::NPT + idx) * S::ES];
    v += T.V[tqi][a] * yvv;
    dt += T.D[tqi][a] * yvv;
    dr += T.V[tqi][a] * L[((base + 1) * S::NPT + idx) * S::ES];
    if constexpr (DIM == 3) dz += T.V[tqi][a] * L[((base + 2) * S::NPT + idx) * S::ES];
  }
  r.v = v;
  r.d[0] = dt;
  r.d[1] = dr;
  if constexpr (DIM == 3) r.d[2] = dz;
#pragma unroll
  for (int e = 0; e < DIM; ++e) r.dd[e] = 0;
}

// value-only field (history, force): single slot per component, stage z and r
// fold into values; theta stage here
template <typename Real, int DIM, int N>
__device__ inline Real eval_stage_t_value(const Tab1D<Real, N>& T, const Real* L, int slot, int tqi, int tqj,
                                          int q) {
  using S = Shape<Real, DIM, N>;
  Real v = 0;
#pragma unroll
  for (int a = 0; a < N; ++a) v += T.V[tqi][a] * L[(slot * S::NPT + q * S::PLANE + tqj * N + a) * S::ES];
  return v;
}

// ---------------------------------------------------------------------------
// Polar geometry at a volume quadrature point
// ---------------------------------------------------------------------------
template <typename Real>
struct PtGeom {
  Real c, s;       // cos, sin of theta
  Real r, inv_r;
  Real inv_dr;     // 1 / dr
  Real inv_rdth;   // 1 / (r dtheta)
  Real inv_dz;
  Real jxw;
  // products of the above used by the transformations below
  Real a1, a2, b1, b2;          // c / dr, s / dr, c / (r dtheta), s / (r dtheta)
  Real l_rr, l_r, l_tt, l_zz;   // Laplacian weights of the reference derivatives
  Real jr1, jr2, jt1, jt2, jz;  // JxW times a1, a2, b1, b2, 1 / dz

  __device__ inline void complete() {
    a1 = c * inv_dr;
    a2 = s * inv_dr;
    b1 = c * inv_rdth;
    b2 = s * inv_rdth;
    l_rr = inv_dr * inv_dr;
    l_r = inv_dr * inv_r;
    l_tt = inv_rdth * inv_rdth;
    l_zz = inv_dz * inv_dz;
    jr1 = jxw * a1;
    jr2 = jxw * a2;
    jt1 = jxw * b1;
    jt2 = jxw * b2;
    jz = jxw * inv_dz;
  }
};

template <typename Real, int DIM, int N>
__device__ inline PtGeom<Real> point_geom(const Geom<Real>& G, const Tab1D<Real, N>& T, const CellId& C, int tqi,
                                          int tqj, int q) {
  PtGeom<Real> g;
  const Real* tr = G.trig + (((size_t)(C.dom ? G.nth[0] : 0) + C.ct) * N + tqi) * 2;
  g.c = tr[0];
  g.s = tr[1];
  const Real dr = pick(C.dom, G.dr);
  g.r = pick(C.dom, G.r0) + dr * (Real(C.cr) + T.x[tqj]);
  g.inv_r = Real(1) / g.r;
  g.inv_dr = Real(1) / dr;
  const Real dth = pick(C.dom, G.dthd);
  g.inv_rdth = g.inv_r / dth;
  g.inv_dz = (DIM == 3) ? Real(1) / G.dz : Real(0);
  Real w = T.w[tqi] * T.w[tqj] * g.r * dth * dr;
  if constexpr (DIM == 3) w *= T.w[q] * G.dz;
  g.jxw = w;
  g.complete();
  return g;
}

// reference derivatives -> Cartesian gradient and Laplacian (exact polar map)
template <typename Real, int DIM>
__device__ inline void to_physical(const PtGeom<Real>& g, const Real* dz_scale, const RefVal<Real, DIM>& rv,
                                   Real (&grad)[DIM], Real& lap, bool want_lap) {
  // d/dr = d1 / dr, (1/r) d/dtheta = d0 / (r dtheta); x = r cos, y = r sin
  grad[0] = g.a1 * rv.d[1] - g.b2 * rv.d[0];
  grad[1] = g.a2 * rv.d[1] + g.b1 * rv.d[0];
  if constexpr (DIM == 3) grad[2] = rv.d[2] * g.inv_dz;
  if (want_lap) {
    // u_rr + u_r / r + u_tt / r^2 (+ u_zz)
    lap = rv.dd[1] * g.l_rr + rv.d[1] * g.l_r + rv.dd[0] * g.l_tt;
    if constexpr (DIM == 3) lap += rv.dd[2] * g.l_zz;
  }
  (void)dz_scale;
}

// physical test coefficients (value g0, gradient G) -> reference ones times JxW
template <typename Real, int DIM>
__device__ inline void to_reference(const PtGeom<Real>& g, Real g0, const Real (&Gp)[DIM], Real* f) {
  f[0] = g.jxw * g0;
  f[1] = g.jt1 * Gp[1] - g.jt2 * Gp[0];                  // theta
  f[2] = g.jr1 * Gp[0] + g.jr2 * Gp[1];                  // r
  if constexpr (DIM == 3) f[3] = g.jz * Gp[2];           // z
}

// Iso-parametric point geometry (metric of the Q_k interpolant of the node
// positions, stored per point, IsoLayout): K[p][m] = d xi_p / d x_m, JxW,
// the mapping term b of the Laplacian and G = K K^T formed here.
template <typename Real, int DIM>
struct IsoPt {
  Real K[DIM][DIM];
  Real jxw;
  Real b[DIM];
  Real G[DIM][DIM];

  __device__ inline void load(const Real* p) {
    using IL = IsoLayout<DIM>;
#pragma unroll
    for (int a = 0; a < DIM; ++a)
#pragma unroll
      for (int m = 0; m < DIM; ++m) K[a][m] = p[IL::K + a * DIM + m];
    jxw = p[IL::JXW];
#pragma unroll
    for (int a = 0; a < DIM; ++a) b[a] = p[IL::B + a];
#pragma unroll
    for (int a = 0; a < DIM; ++a)
#pragma unroll
      for (int c = a; c < DIM; ++c) {
        Real t = 0;
#pragma unroll
        for (int m = 0; m < DIM; ++m) t += K[a][m] * K[c][m];
        G[a][c] = G[c][a] = t;
      }
  }
};

// reference values with the mixed second derivatives, which a general
// metric couples: mx = {theta r, theta z, r z}
template <typename Real, int DIM>
struct RefValX {
  Real v;
  Real d[DIM];
  Real dd[DIM];
  Real mx[3];
};

// reference derivatives -> Cartesian gradient and Laplacian (general metric)
template <typename Real, int DIM>
__device__ inline void to_physical(const IsoPt<Real, DIM>& g, const Real*, const RefValX<Real, DIM>& rv,
                                   Real (&grad)[DIM], Real& lap, bool want_lap) {
#pragma unroll
  for (int m = 0; m < DIM; ++m) {
    Real t = 0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) t += g.K[a][m] * rv.d[a];
    grad[m] = t;
  }
  if (want_lap) {
    Real l = 2 * g.G[0][1] * rv.mx[0];
    if constexpr (DIM == 3) l += 2 * (g.G[0][2] * rv.mx[1] + g.G[1][2] * rv.mx[2]);
#pragma unroll
    for (int a = 0; a < DIM; ++a) l += g.G[a][a] * rv.dd[a] - g.b[a] * rv.d[a];
    lap = l;
  }
}

// physical test coefficients -> reference ones times JxW (general metric)
template <typename Real, int DIM>
__device__ inline void to_reference(const IsoPt<Real, DIM>& g, Real g0, const Real (&Gp)[DIM], Real* f) {
  f[0] = g.jxw * g0;
  Real w[DIM];
#pragma unroll
  for (int m = 0; m < DIM; ++m) w[m] = g.jxw * Gp[m];
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    Real t = 0;
#pragma unroll
    for (int m = 0; m < DIM; ++m) t += g.K[a][m] * w[m];
    f[1 + a] = t;
  }
}

// Pointwise linearized operator at one volume point (Sec. 2.3 blocks):
// reference values/derivatives of the increment (rv velocity, rp pressure)
// and the stored linearization lv -> reference test coefficients times JxW,
// tc[comp][{value, theta, r, z}].
//   g_v = c_t du + (grad u) du + (grad du) a,   R' du = g_v - nu lap du + grad dp
//   G_v = nu grad du - dp I + tau R' du (x) a + tau R (x) du,  g_q = div du,  G_q = tau R' du
// (GeoT, RV: polar PtGeom with RefVal, or IsoPt with RefValX.)
template <typename Real, int DIM, typename GeoT, typename RV>
__device__ inline void pointwise_jacobian(const GeoT& g, const RV (&rv)[DIM], const RV& rp, const Real* lv, Real nu,
                                          Real ct, Real (&tc)[DIM + 1][DIM + 1]) {
  using LL = LinLayout<DIM>;
  Real du[DIM], gdu[DIM][DIM], ldu[DIM], gdp[DIM], dummy;
#pragma unroll
  for (int m = 0; m < DIM; ++m) {
    du[m] = rv[m].v;
    to_physical<Real, DIM>(g, nullptr, rv[m], gdu[m], ldu[m], true);
  }
  to_physical<Real, DIM>(g, nullptr, rp, gdp, dummy, false);
  const Real dp = rp.v;
  Real a[DIM], gu[DIM][DIM], tR[DIM];
#pragma unroll
  for (int m = 0; m < DIM; ++m) {
    a[m] = lv[LL::A + m];
    tR[m] = lv[LL::TR + m];
#pragma unroll
    for (int e = 0; e < DIM; ++e) gu[m][e] = lv[LL::GU + m * DIM + e];
  }
  const Real tau = lv[LL::TAU];
  Real gv[DIM], Rp[DIM], divdu = 0;
#pragma unroll
  for (int m = 0; m < DIM; ++m) {
    Real s2 = ct * du[m];
#pragma unroll
    for (int e = 0; e < DIM; ++e) s2 += gu[m][e] * du[e] + gdu[m][e] * a[e];
    gv[m] = s2;
    Rp[m] = s2 - nu * ldu[m] + gdp[m];
    divdu += gdu[m][m];
  }
#pragma unroll
  for (int m = 0; m < DIM; ++m) {
    Real Gm[DIM];
    const Real tRp = tau * Rp[m];
#pragma unroll
    for (int e = 0; e < DIM; ++e) Gm[e] = nu * gdu[m][e] + tRp * a[e] + tR[m] * du[e];
    Gm[m] -= dp;
    to_reference<Real, DIM>(g, gv[m], Gm, tc[m]);
  }
  Real Gq[DIM];
#pragma unroll
  for (int e = 0; e < DIM; ++e) Gq[e] = tau * Rp[e];
  to_reference<Real, DIM>(g, divdu, Gq, tc[DIM]);
}

// ---------------------------------------------------------------------------
// Integration: test coefficients in LDS slots comp*NT + {0: value, 1: theta,
// 2: r, 3: z} at point [q][qj][qi] -> nodal line of the lane, stored into the
// local-result buffer E[comp][local node][cell] (cell fastest; no atomics:
// the per-node sum over cells is done by k_gather in a fixed order).
// ---------------------------------------------------------------------------
template <typename Real, int DIM, int N>
__device__ inline void integrate_store(const Tab1D<Real, N>& T, const Tab1D<Real, N>& Tz, Real* L, int ta, int tb,
                                       bool active, int cell, long long ncells, Real* __restrict__ E) {
  using S = Shape<Real, DIM, N>;
  constexpr int NZ = S::NZ, NC = S::NC, NT = S::NT;
  constexpr int NX = (DIM == 3) ? 3 : 2;
  // theta stage: lane (ta, tqj=tb) contracts over qi
  Real X[NC][NX][NZ];
  if (active) {
#pragma unroll
    for (int m = 0; m < NC; ++m)
#pragma unroll
      for (int q = 0; q < NZ; ++q) {
        Real x0 = 0, xr = 0, xz = 0;
#pragma unroll
        for (int qi = 0; qi < N; ++qi) {
          const int idx = q * S::PLANE + tb * N + qi;
          x0 += T.V[qi][ta] * L[((m * NT + 0) * S::NPT + idx) * S::ES] + T.D[qi][ta] * L[((m * NT + 1) * S::NPT + idx) * S::ES];
          xr += T.V[qi][ta] * L[((m * NT + 2) * S::NPT + idx) * S::ES];
          if constexpr (DIM == 3) xz += T.V[qi][ta] * L[((m * NT + 3) * S::NPT + idx) * S::ES];
        }
        X[m][0][q] = x0;
        X[m][1][q] = xr;
        if constexpr (DIM == 3) X[m][2][q] = xz;
      }
  }
  __syncthreads();
  if (active) {
#pragma unroll
    for (int m = 0; m < NC; ++m)
#pragma unroll
      for (int j = 0; j < NX; ++j)
#pragma unroll
        for (int q = 0; q < NZ; ++q) L[((m * NX + j) * S::NPT + q * S::PLANE + tb * N + ta) * S::ES] = X[m][j][q];
  }
  __syncthreads();
  if (!active) return;
  // r stage: lane (ta, tb) contracts over qj; z stage in registers
  Real* Ec = E + cell;
#pragma unroll
  for (int m = 0; m < NC; ++m) {
    Real Y0[NZ], Yz[NZ];
#pragma unroll
    for (int q = 0; q < NZ; ++q) {
      Real y0 = 0, yz = 0;
#pragma unroll
      for (int qj = 0; qj < N; ++qj) {
        const int idx = q * S::PLANE + qj * N + ta;
        y0 += T.V[qj][tb] * L[((m * NX + 0) * S::NPT + idx) * S::ES] + T.D[qj][tb] * L[((m * NX + 1) * S::NPT + idx) * S::ES];
        if constexpr (DIM == 3) yz += T.V[qj][tb] * L[((m * NX + 2) * S::NPT + idx) * S::ES];
      }
      Y0[q] = y0;
      Yz[q] = yz;
    }
#pragma unroll
    for (int c = 0; c < NZ; ++c) {
      Real o;
      if constexpr (DIM == 3) {
        o = 0;
#pragma unroll
        for (int q = 0; q < NZ; ++q) o += Tz.V[q][c] * Y0[q] + Tz.D[q][c] * Yz[q];
      } else {
        o = Y0[0];
      }
      Ec[(size_t)(m * S::NPT + c * S::PLANE + tb * N + ta) * ncells] = o;
    }
  }
}

// ---------------------------------------------------------------------------
// Gather: dst[node] = sum of the local results of every cell (and, on the
// interface, every mortar cell side) that contains the node, in a fixed order;
// constrained rows: mode 0 dst = src, mode 1 dst = 0.  One lane per node.
// ---------------------------------------------------------------------------
template <typename Real, int DIM, int N>
__device__ inline void gather_node(const Geom<Real>& G, int k, const Real* __restrict__ E,
                                   const Real* __restrict__ Em, const Real* __restrict__ src,
                                   Real* __restrict__ dst, int mode, int strip, long long g) {
  using S = Shape<Real, DIM, N>;
  constexpr int NC = S::NC;
  const long long nnodes = G.ndofs / NC;
  if (g >= nnodes) return;
  const int dom = g >= G.node_off1;
  const long long l = g - (dom ? G.node_off1 : 0);
  const int ntn = pick(dom, G.ntd), ntc = pick(dom, G.nth);
  const int it = (int)(l % ntn);
  const long long l2 = l / ntn;
  const int nrn = pick(dom, G.nrn), nrd = pick(dom, G.nr);
  const int ir = (int)(l2 % nrn);
  const int iz = (int)(l2 / nrn);
  // candidate cells per direction: (cell index, local node index, valid);
  // the loops below have fixed trip counts so that all loads are issued
  // together (invalid candidates are predicated off)
  int tc[2], ta[2];
  bool tv[2];
  tc[0] = it / k;
  ta[0] = it % k;
  tv[0] = true;
  tc[1] = (tc[0] == 0 ? ntc : tc[0]) - 1;
  ta[1] = k;
  tv[1] = ta[0] == 0;
  int rc[2], rb[2];
  bool rv[2];
  rc[0] = ir / k;
  rb[0] = ir % k;
  rv[0] = rc[0] < nrd;
  rc[1] = ir / k - 1;
  rb[1] = k;
  rv[1] = (ir % k == 0) && ir > 0;
  int zc[2], zb[2];
  bool zv[2];
  if constexpr (DIM == 3) {
    zc[0] = iz / k;
    zb[0] = iz % k;
    zv[0] = zc[0] < G.nz;
    zc[1] = iz / k - 1;
    zb[1] = k;
    zv[1] = (iz % k == 0) && iz > 0;
  } else {
    zc[0] = zc[1] = 0;
    zb[0] = zb[1] = 0;
    zv[0] = true;
    zv[1] = false;
  }
  Real acc[NC];
#pragma unroll
  for (int m = 0; m < NC; ++m) acc[m] = 0;
  const int cbase = dom ? (int)G.cell_off1 : 0;
  const size_t cstride = (size_t)S::NPT * G.ncells;
  Real cv[2][2][2][NC];  // candidate contributions [z][r][theta][comp]
  if (strip) {
    // strip layout of the quad volume kernel: batches of 16 theta-consecutive
    // cells, 16 k + 1 node columns per (comp, z, r) node position; a node on a
    // batch boundary appears in two batches (last column of the earlier one)
    const int S16 = 16 * k, nbt = ntc / 16;
    const size_t nblk = (size_t)(G.ncells / 16), pstride = nblk * S16;
    const Real* Eb = E + (size_t)N * N * NC * pstride;  // last columns of the batches
    int sb[2], sj[2];
    bool sv[2];
    sb[0] = it / S16;
    sj[0] = it % S16;
    sv[0] = true;
    sb[1] = (sb[0] == 0 ? nbt : sb[0]) - 1;
    sj[1] = S16;
    sv[1] = sj[0] == 0;
    // every candidate's loads are issued before any of them is summed (an
    // accumulation inside each candidate's branch waits for that branch's
    // loads, one memory round trip per candidate); the sum keeps the fixed
    // candidate order
#pragma unroll
    for (int z = 0; z < 2; ++z)
#pragma unroll
      for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int t = 0; t < 2; ++t) {
#pragma unroll
          for (int m = 0; m < NC; ++m) cv[z][r][t][m] = 0;
          if (!(zv[z] && rv[r] && sv[t])) continue;
          const int ring = (cbase + ntc * (rc[r] + nrd * zc[z])) / 16;
          const size_t pos = (size_t)(zb[z] * N + rb[r]);
          const size_t st = t == 0 ? pstride : nblk;
          const Real* e = t == 0 ? E + pos * pstride + (size_t)(ring + sb[0]) * S16 + sj[0]
                                 : Eb + pos * nblk + (ring + sb[1]);
#pragma unroll
          for (int m = 0; m < NC; ++m) cv[z][r][t][m] = e[(size_t)m * N * N * st];
        }
  } else {
#pragma unroll
    for (int z = 0; z < 2; ++z)
#pragma unroll
      for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int t = 0; t < 2; ++t) {
#pragma unroll
          for (int m = 0; m < NC; ++m) cv[z][r][t][m] = 0;
          if (!(zv[z] && rv[r] && tv[t])) continue;
          const int cell = cbase + tc[t] + ntc * (rc[r] + nrd * zc[z]);
          const int loc = (DIM == 3 ? zb[z] * S::PLANE : 0) + rb[r] * N + ta[t];
          const Real* e = E + (size_t)loc * G.ncells + cell;
#pragma unroll
          for (int m = 0; m < NC; ++m) cv[z][r][t][m] = e[m * cstride];
        }
  }
  // mortar cell sides: every node of a rotor outer-ring cell or a stator
  // inner-ring cell (the grad v face term reaches all of them)
  int bm = -1;
  if (dom == 0 && ir >= k * (G.nr[0] - 1)) bm = ir - k * (G.nr[0] - 1);
  if (dom == 1 && ir <= k) bm = ir;
  Real mv[2][2][NC];  // mortar contributions [z][theta][comp], loaded before any sum
#pragma unroll
  for (int z = 0; z < 2; ++z)
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int m = 0; m < NC; ++m) mv[z][t][m] = 0;
  if (bm >= 0 && Em) {
    // face sides: the rotor's n_theta[0] n_z faces, then the stator's
    const int nf0 = G.nth[0] * G.nz;
    const int nsides = nf0 + G.nth[1] * G.nz;
    const size_t mstride = (size_t)S::NPT * nsides;
#pragma unroll
    for (int z = 0; z < 2; ++z)
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        if (!(zv[z] && tv[t])) continue;
        const int cs = (dom ? nf0 : 0) + tc[t] + ntc * zc[z];
        const int loc = (DIM == 3 ? zb[z] * S::PLANE : 0) + bm * N + ta[t];
        const Real* e = Em + (size_t)loc * nsides + cs;
#pragma unroll
        for (int m = 0; m < NC; ++m) mv[z][t][m] = e[m * mstride];
      }
  }
#pragma unroll
  for (int z = 0; z < 2; ++z)
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int m = 0; m < NC; ++m) acc[m] += cv[z][r][t][m];
#pragma unroll
  for (int z = 0; z < 2; ++z)
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int m = 0; m < NC; ++m) acc[m] += mv[z][t][m];
  const bool vf = vel_fixed<Real, DIM>(G, dom, ir, iz);
  const bool pf = p_fixed(G, dom, it, ir, iz);
  Real* d = dst + g * NC;
  const Real* sv = src + g * NC;
#pragma unroll
  for (int m = 0; m < NC; ++m) {
    const bool fixed = m < DIM ? vf : pf;
    d[m] = fixed ? (mode == 0 ? sv[m] : Real(0)) : acc[m];
  }
}

template <typename Real, int DIM, int N>
__global__ __launch_bounds__(256) void k_gather(Geom<Real> G, int k, const Real* __restrict__ E,
                                                const Real* __restrict__ Em, const Real* __restrict__ src,
                                                Real* __restrict__ dst, int mode, int strip) {
  gather_node<Real, DIM, N>(G, k, E, Em, src, dst, mode, strip, (long long)blockIdx.x * blockDim.x + threadIdx.x);
}

// lane's nodal line of a vector (all components), constrained entries as zero
// when mask is set
template <typename Real, int DIM, int N, typename In>
__device__ inline void gather_line(const Geom<Real>& G, int k, const CellId& C, int ta, int tb,
                                   const In* __restrict__ v, bool mask, Real (*u)[Shape<Real, DIM, N>::NZ]) {
  using S = Shape<Real, DIM, N>;
#pragma unroll
  for (int c = 0; c < S::NZ; ++c) {
    int it, ir, iz;
    const long long node = node_of<Real, DIM>(G, k, C, ta, tb, c, it, ir, iz);
    const bool vf = mask && vel_fixed<Real, DIM>(G, C.dom, ir, iz);
    const bool pf = mask && p_fixed(G, C.dom, it, ir, iz);
    // load unconditionally so the loads of all nodes are in flight together
    Real w[S::NC];
#pragma unroll
    for (int m = 0; m < S::NC; ++m) w[m] = Real(v[node * S::NC + m]);
#pragma unroll
    for (int m = 0; m < DIM; ++m) u[m][c] = vf ? Real(0) : w[m];
    u[DIM][c] = pf ? Real(0) : w[DIM];
  }
}

// ---------------------------------------------------------------------------
// Jacobian vmult with stored linearization (Sec. 2.3 blocks, volume part)
// ---------------------------------------------------------------------------
template <typename Real, int DIM, int N, bool ISO = false>
struct PlaneShape {
  static constexpr int ZS = (DIM == 3) ? 3 * DIM + 2 : DIM + 1;  // z-stage arrays (velocity V,D,DD; pressure V,D)
  // r-stage outputs per velocity component: V, D, DD of the z value, V of the
  // z derivative and second derivative, and (iso-parametric, 3D) D of the z
  // derivative for the mixed r z derivative
  static constexpr int NYV = (DIM == 3) ? (ISO ? 6 : 5) : 3;
  static constexpr int YS = (DIM == 3) ? NYV * DIM + 3 : 3 * DIM + 2; // r-stage arrays
  static constexpr int TS = (DIM + 1) * (DIM + 1);                  // test coefficients
  static constexpr int XS = (DIM + 1) * ((DIM == 3) ? 3 : 2);       // theta-transposed test arrays
  static constexpr int A = (ZS > TS ? ZS : TS) * N * N;             // doubles per cell in buffer A
  static constexpr int B = (YS > XS ? YS : XS) * N * N;             // doubles per cell in buffer B
  static constexpr int REGION = A + B;
};

// Jacobian vmult with stored linearization, volume part (Sec. 2.3 blocks).
// Plane pipeline: for every z plane q of Gauss points the lanes run the z
// contraction of their nodal line for that plane, the r and theta
// contractions through LDS, the pointwise operator, and the transposed theta
// and r contractions; the z part of the integration accumulates in registers.
// LDS holds one plane per cell in two ping-pong buffers.
template <typename Real, int DIM, int N, bool ISO = false>
struct VolumeSmem {
  Tab1D<Real, N> sT;
  Real lds[Shape<Real, DIM, N>::CPW * PlaneShape<Real, DIM, N, ISO>::REGION];
};

// ISO: iso-parametric cells (per-point metric G.geo, mixed second
// derivatives of the increment's velocity in the Laplacian)
template <typename Real, int DIM, int N, bool ISO = false>
__device__ __attribute__((always_inline)) inline void volume_block(const Geom<Real>& G, const Tab1D<Real, N>& T, int k, int vblock,
                                    const Real* __restrict__ lin, const Real* __restrict__ src,
                                    Real* __restrict__ E, VolumeSmem<Real, DIM, N, ISO>& sm) {
  using S = Shape<Real, DIM, N>;
  using P = PlaneShape<Real, DIM, N, ISO>;
  constexpr int NYV = P::NYV;
  using LL = LinLayout<DIM>;
  constexpr int NZ = S::NZ, NC = S::NC, PL = N * N;
  Real* lds = sm.lds;
  Tab1D<Real, N>& sT = sm.sT;
  const int lane = threadIdx.x;
  {
    constexpr int NW = (int)(sizeof(Tab1D<Real, N>) / sizeof(Real));
    const Real* tw = (const Real*)&T;
    for (int i = lane; i < NW; i += 64) ((Real*)&sT)[i] = tw[i];
  }
  const int cl = lane / S::TPC;
  const int t = lane % S::TPC;
  const int ta = t % N, tb = t / N;
  const int cell = vblock * S::CPW + cl;
  const bool active = cl < S::CPW && cell < G.ncells;
  Real* A = lds + (active ? cl : 0) * P::REGION;
  Real* B = A + P::A;
  const CellId C = decode_cell(G, active ? cell : 0);
  const int me = tb * N + ta;  // this lane's position in a plane
  // z-stage outputs and theta-transposed test arrays are written transposed
  // (theta index major) so that every later LDS read is contiguous
  const int meT = ta * N + tb;

  Real u[NC][NZ];
  if (active) gather_line<Real, DIM, N>(G, k, C, ta, tb, src, true, u);
  Real o[NC][NZ];
#pragma unroll
  for (int m = 0; m < NC; ++m)
#pragma unroll
    for (int c = 0; c < NZ; ++c) o[m][c] = 0;
  Real lv[LL::SIZE];
  const Real* lbase = lin + ((size_t)(active ? cell : 0) * S::NPT + me) * LL::SIZE;
  if (active)
#pragma unroll
    for (int j = 0; j < LL::SIZE; ++j) lv[j] = lbase[j];
  const Real nu = G.nu, ct = G.ct;

#pragma unroll
  for (int q = 0; q < NZ; ++q) {
    // iso-parametric metric of the lane's point in plane q, requested before
    // the z and r stages so that its latency overlaps them (3D degree 4:
    // requested at the theta stage, where the registers allow it)
    constexpr bool kEarlyGeo = ISO && (DIM == 2 || N <= 4);
    Real gq[kEarlyGeo ? IsoLayout<DIM>::SIZE : 1];
    if constexpr (kEarlyGeo) {
      if (active) {
        const Real* gp = G.geo + ((size_t)cell * S::NPT + q * PL + me) * IsoLayout<DIM>::SIZE;
#pragma unroll
        for (int j = 0; j < IsoLayout<DIM>::SIZE; ++j) gq[j] = gp[j];
      }
    }
    // ---- z stage for plane q (registers) -> A
    if (active) {
#pragma unroll
      for (int m = 0; m < NC; ++m) {
        const bool vel = m < DIM;
        const int base = vel ? m * (DIM == 3 ? 3 : 1) : DIM * (DIM == 3 ? 3 : 1);
        if constexpr (DIM == 3) {
          Real sv = 0, sd = 0, sdd = 0;
#pragma unroll
          for (int c = 0; c < NZ; ++c) {
            sv += T.V[q][c] * u[m][c];
            sd += T.D[q][c] * u[m][c];
            if (vel) sdd += T.DD[q][c] * u[m][c];
          }
          A[(base + 0) * PL + meT] = sv;
          A[(base + 1) * PL + meT] = sd;
          if (vel) A[(base + 2) * PL + meT] = sdd;
        } else {
          A[base * PL + meT] = u[m][0];
        }
      }
    }
    __syncthreads();
    // ---- r stage: lane (ta, tqj = tb) reads column ta of A -> B.  All reads
    // are issued before any store so they overlap (A and B may alias as far
    // as the compiler can tell).
    if (active) {
      constexpr int ZV = (DIM == 3) ? 3 : 1, ZP = (DIM == 3) ? 2 : 1;
      Real zin[P::ZS][N];
#pragma unroll
      for (int arr = 0; arr < P::ZS; ++arr)
#pragma unroll
        for (int b = 0; b < N; ++b) zin[arr][b] = A[arr * PL + ta * N + b];
      Real yout[P::YS];
#pragma unroll
      for (int m = 0; m < NC; ++m) {
        const bool vel = m < DIM;
        const int zb = vel ? m * ZV : DIM * ZV;
        const int yb = vel ? m * NYV : DIM * NYV;
        Real vv = 0, dv = 0, ddv = 0, vd = 0, vdd = 0, dvd = 0;
#pragma unroll
        for (int b = 0; b < N; ++b) {
          const Real zv = zin[zb][b];
          vv += sT.V[tb][b] * zv;
          dv += sT.D[tb][b] * zv;
          if (vel) ddv += sT.DD[tb][b] * zv;
          if constexpr (DIM == 3) {
            vd += sT.V[tb][b] * zin[zb + 1][b];
            if (vel) vdd += sT.V[tb][b] * zin[zb + 2][b];
            if (ISO && vel) dvd += sT.D[tb][b] * zin[zb + 1][b];
          }
        }
        yout[yb + 0] = vv;
        yout[yb + 1] = dv;
        if constexpr (DIM == 3) {
          if (vel) {
            yout[yb + 2] = ddv;
            yout[yb + 3] = vd;
            yout[yb + 4] = vdd;
            if constexpr (ISO) yout[yb + 5] = dvd;
          } else {
            yout[yb + 2] = vd;
          }
        } else {
          if (vel) yout[yb + 2] = ddv;
        }
      }
      (void)ZP;
#pragma unroll
      for (int arr = 0; arr < P::YS; ++arr) B[arr * PL + me] = yout[arr];
    }
    __syncthreads();
    // ---- theta stage + pointwise operator: lane (tqi = ta, tqj = tb) -> test coefficients in A
    Real lnext[LL::SIZE];
    if (active && q + 1 < NZ)
#pragma unroll
      for (int j = 0; j < LL::SIZE; ++j) lnext[j] = lbase[(q + 1) * PL * LL::SIZE + j];
    if (active) {
      using RV = std::conditional_t<ISO, RefValX<Real, DIM>, RefVal<Real, DIM>>;
      RV rv[DIM], rp;
#pragma unroll
      for (int m = 0; m < DIM; ++m) {
        const Real* y = B + m * NYV * PL + tb * N;
        Real v = 0, dt = 0, ddt = 0, dr = 0, ddr = 0, dz = 0, ddz = 0, dtr = 0, dtz = 0, drz = 0;
#pragma unroll
        for (int a2 = 0; a2 < N; ++a2) {
          const Real yvv = y[a2];
          v += sT.V[ta][a2] * yvv;
          dt += sT.D[ta][a2] * yvv;
          ddt += sT.DD[ta][a2] * yvv;
          dr += sT.V[ta][a2] * y[1 * PL + a2];
          ddr += sT.V[ta][a2] * y[2 * PL + a2];
          if constexpr (ISO) dtr += sT.D[ta][a2] * y[1 * PL + a2];
          if constexpr (DIM == 3) {
            dz += sT.V[ta][a2] * y[3 * PL + a2];
            ddz += sT.V[ta][a2] * y[4 * PL + a2];
            if constexpr (ISO) {
              dtz += sT.D[ta][a2] * y[3 * PL + a2];
              drz += sT.V[ta][a2] * y[5 * PL + a2];
            }
          }
        }
        if constexpr (ISO) {
          rv[m].mx[0] = dtr;
          rv[m].mx[1] = dtz;
          rv[m].mx[2] = drz;
        }
        rv[m].v = v;
        rv[m].d[0] = dt;
        rv[m].d[1] = dr;
        rv[m].dd[0] = ddt;
        rv[m].dd[1] = ddr;
        if constexpr (DIM == 3) {
          rv[m].d[2] = dz;
          rv[m].dd[2] = ddz;
        }
      }
      {
        const Real* y = B + DIM * NYV * PL + tb * N;
        Real v = 0, dt = 0, dr = 0, dz = 0;
#pragma unroll
        for (int a2 = 0; a2 < N; ++a2) {
          v += sT.V[ta][a2] * y[a2];
          dt += sT.D[ta][a2] * y[a2];
          dr += sT.V[ta][a2] * y[1 * PL + a2];
          if constexpr (DIM == 3) dz += sT.V[ta][a2] * y[2 * PL + a2];
        }
        rp.v = v;
        rp.d[0] = dt;
        rp.d[1] = dr;
        if constexpr (DIM == 3) rp.d[2] = dz;
#pragma unroll
        for (int e = 0; e < DIM; ++e) rp.dd[e] = 0;
        if constexpr (ISO) rp.mx[0] = rp.mx[1] = rp.mx[2] = 0;
      }
      Real tc[NC][S::NT];
      if constexpr (ISO) {
        IsoPt<Real, DIM> g;
        if constexpr (kEarlyGeo) g.load(gq);
        else g.load(G.geo + ((size_t)cell * S::NPT + q * PL + me) * IsoLayout<DIM>::SIZE);
        pointwise_jacobian<Real, DIM>(g, rv, rp, lv, nu, ct, tc);
      } else {
        const PtGeom<Real> g = point_geom<Real, DIM, N>(G, sT, C, ta, tb, q);
        pointwise_jacobian<Real, DIM>(g, rv, rp, lv, nu, ct, tc);
      }
#pragma unroll
      for (int m = 0; m < NC; ++m)
#pragma unroll
        for (int j = 0; j < S::NT; ++j) A[(m * S::NT + j) * PL + me] = tc[m][j];
    }
    if (active && q + 1 < NZ)
#pragma unroll
      for (int j = 0; j < LL::SIZE; ++j) lv[j] = lnext[j];
    __syncthreads();
    // ---- theta transpose: lane (ta, tqj = tb) contracts over qi -> B (all
    // reads first, then the stores)
    constexpr int NX = (DIM == 3) ? 3 : 2;
    if (active) {
      Real tin[P::TS][N];
#pragma unroll
      for (int arr = 0; arr < P::TS; ++arr)
#pragma unroll
        for (int qi = 0; qi < N; ++qi) tin[arr][qi] = A[arr * PL + tb * N + qi];
      Real xout[P::XS];
#pragma unroll
      for (int m = 0; m < NC; ++m) {
        const Real(*tp)[N] = tin + m * S::NT;
        Real x0 = 0, xr = 0, xz = 0;
#pragma unroll
        for (int qi = 0; qi < N; ++qi) {
          x0 += sT.V[qi][ta] * tp[0][qi] + sT.D[qi][ta] * tp[1][qi];
          xr += sT.V[qi][ta] * tp[2][qi];
          if constexpr (DIM == 3) xz += sT.V[qi][ta] * tp[3][qi];
        }
        xout[m * NX + 0] = x0;
        xout[m * NX + 1] = xr;
        if constexpr (DIM == 3) xout[m * NX + 2] = xz;
      }
#pragma unroll
      for (int arr = 0; arr < P::XS; ++arr) B[arr * PL + meT] = xout[arr];
    }
    __syncthreads();
    // ---- r transpose: lane (ta, tb) contracts over qj; z part accumulates
    if (active) {
#pragma unroll
      for (int m = 0; m < NC; ++m) {
        Real y0 = 0, yz = 0;
#pragma unroll
        for (int qj = 0; qj < N; ++qj) {
          const int xi = ta * N + qj;
          y0 += sT.V[qj][tb] * B[(m * NX + 0) * PL + xi] + sT.D[qj][tb] * B[(m * NX + 1) * PL + xi];
          if constexpr (DIM == 3) yz += sT.V[qj][tb] * B[(m * NX + 2) * PL + xi];
        }
        if constexpr (DIM == 3) {
#pragma unroll
          for (int c = 0; c < NZ; ++c) o[m][c] += T.V[q][c] * y0 + T.D[q][c] * yz;
        } else {
          o[m][0] = y0;
        }
      }
    }
  }
  if (!active) return;
  Real* Ec = E + cell;
#pragma unroll
  for (int m = 0; m < NC; ++m)
#pragma unroll
    for (int c = 0; c < NZ; ++c) Ec[(size_t)(m * S::NPT + c * PL + me) * G.ncells] = o[m][c];
}

template <typename Real, int DIM, int N, bool ISO = false>
__global__ __launch_bounds__(64) void k_jacobian_volume(Geom<Real> G, Tab1D<Real, N> T, int k,
                                                                     const Real* __restrict__ lin,
                                                                     const Real* __restrict__ src,
                                                                     Real* __restrict__ E) {
  __shared__ VolumeSmem<Real, DIM, N, ISO> sm;
  volume_block<Real, DIM, N, ISO>(G, T, k, blockIdx.x, lin, src, E, sm);
}

// ---------------------------------------------------------------------------
// Jacobian vmult, volume part, quad layout (3D, N <= 4).  A quad of four
// lanes owns one cell: lane t holds the theta-slice t of the cell's nodes
// (all r and z positions).  The z and r contractions run in registers; the
// theta contractions exchange values inside the quad with DPP quad
// permutations, so the sum factorization needs no LDS.  With N = 3 the
// fourth lane of a quad duplicates the last slice and stores nothing; every
// lane runs every instruction so the cross-lane reads always see live data.
// ---------------------------------------------------------------------------
template <typename Real, int N>
struct QuadShape {
  static constexpr int CPW = 16;  // cells per wavefront
  static constexpr int PL = N * N;
  static constexpr int NPT = N * N * N;
};

// DPP quad permutation: lane t of a quad reads lane (t + S) mod N; lanes
// t >= N read what lane N-1 reads, so that they repeat lane N-1 exactly
template <int S, int N>
__device__ constexpr int quad_ctrl() {
  int c = 0;
  for (int t = 0; t < 4; ++t) c |= (((t < N ? t : N - 1) + S) % N) << (2 * t);
  return c;
}

template <int S, int N, typename Real>
__device__ inline Real qshift(Real x) {
  constexpr int ctrl = quad_ctrl<S, N>();
  if constexpr (S == 0) {
    return x;
  } else if constexpr (sizeof(Real) == 8) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), ctrl, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), ctrl, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
  } else {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), ctrl, 0xF, 0xF, true));
  }
}

// the N values of x held by the quad, rotated so that xs[s] is lane t+s's
template <int N, typename Real>
__device__ inline void quad_rotate(Real x, Real (&xs)[N]) {
  xs[0] = x;
  if constexpr (N > 1) xs[1] = qshift<1, N>(x);
  if constexpr (N > 2) xs[2] = qshift<2, N>(x);
  if constexpr (N > 3) xs[3] = qshift<3, N>(x);
}

template <int N, typename Real>
__device__ inline Real quad_dot(const Real (&c)[N], const Real (&xs)[N]) {
  Real v = c[0] * xs[0];
#pragma unroll
  for (int s = 1; s < N; ++s) v += c[s] * xs[s];
  return v;
}

// value of x held by the previous lane of the wavefront (DPP wave shift right
// by one; lane 0 reads 0)
template <typename Real>
__device__ inline Real from_prev_lane(Real x) {
  constexpr int kWaveShr1 = 0x138;
  if constexpr (sizeof(Real) == 8) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), kWaveShr1, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), kWaveShr1, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
  } else {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), kWaveShr1, 0xF, 0xF, true));
  }
}

// value v[t] of a lane-indexed table whose entries are wave-uniform
template <int N, typename Real>
__device__ inline Real lane_select(int t, const Real (&v)[N]) {
  // written as a masked sum: a chain of selects is turned into a table in
  // private (scratch) memory indexed by the lane
  Real r = Real(0);
#pragma unroll
  for (int i = 0; i < N; ++i) r = __builtin_fma(t == i ? Real(1) : Real(0), v[i], r);
  return r;
}

template <typename Real>
__device__ inline void load_node4(const Real* p, Real (&w)[4]) {
  if constexpr (sizeof(Real) == 8) {
    const double2* q = reinterpret_cast<const double2*>(p);
    const double2 a = q[0], b = q[1];
    w[0] = a.x;
    w[1] = a.y;
    w[2] = b.x;
    w[3] = b.y;
  } else {
    const float4 a = *reinterpret_cast<const float4*>(p);
    w[0] = a.x;
    w[1] = a.y;
    w[2] = a.z;
    w[3] = a.w;
  }
}

template <typename Real, int NV>
__device__ inline void load_lin(const Real* p, Real (&w)[NV]) {
  if constexpr (sizeof(Real) == 8) {
    const double2* q = reinterpret_cast<const double2*>(p);
#pragma unroll
    for (int i = 0; i < NV / 2; ++i) {
      const double2 a = q[i];
      w[2 * i] = a.x;
      w[2 * i + 1] = a.y;
    }
  } else {
    const float4* q = reinterpret_cast<const float4*>(p);
#pragma unroll
    for (int i = 0; i < NV / 4; ++i) {
      const float4 a = q[i];
      w[4 * i] = a.x;
      w[4 * i + 1] = a.y;
      w[4 * i + 2] = a.z;
      w[4 * i + 3] = a.w;
    }
  }
}

// The quad kernel works in the collocation basis of the Gauss points: the
// nodal values are first interpolated to the cell's Gauss points (z, r in
// registers, theta across the quad); first and second reference derivatives
// at every point then follow from the Gauss-point derivative matrices CD and
// CDD along each direction.  The transposed steps run in reverse: the test
// coefficients of every point are accumulated in the collocation basis (the
// transposed CD applied along r, z and, across the quad, theta) and finally
// interpolated back to the nodes.
//
// ULDS: the field values at the Gauss points are kept in LDS (4 (k+1)^2
// values per lane: 18 KB per FP64 wavefront at degree 2, 32 KB at degree 3)
// instead of registers and the linearization data of each point is loaded
// when the point starts (no prefetch ring).  That takes the FP64 degree-2
// kernel from about 370 registers per lane to under 256, i.e. from one to two
// wavefronts per SIMD, which hide each other's memory latency.
//
// LINC: linearization source C.  Per point only tau and tau R are read (lin
// then holds 4 values per point, in the point order of the full store); the
// advection velocity a = u - w (w the mesh velocity of rotor cells) and the
// velocity gradient grad u are evaluated from the state's nodal values with
// the same collocation steps as the increment (picard: grad u = 0).  The
// state's point values stay in registers, or in LDS after the increment's
// (3 (k+1)^2 more values per lane) when ULDS is set.
template <typename Real, int N, bool ULDS = false, bool LINC = false>
__device__ __attribute__((always_inline)) inline void volume_quad(const Geom<Real>& G, const Tab1D<Real, N>& T, int k, int vblock,
                                   const Real* __restrict__ lin, const Real* __restrict__ src,
                                   Real* __restrict__ E, bool strip, Real* __restrict__ us = nullptr,
                                   const Real* __restrict__ state = nullptr, int picard = 0) {
  constexpr int DIM = 3, NC = 4, NT = 4;
  using Q = QuadShape<Real, N>;
  using LL = LinLayout<DIM>;
  constexpr int LW = LINC ? 4 : LL::SIZE;  // values read per point
  Real* ss = nullptr;                      // state point values (ULDS and LINC)
  if constexpr (ULDS && LINC) ss = us + NC * N * N * 64;
  static_assert(N <= 4, "quad layout holds at most four theta slices");
  const int lane = threadIdx.x & 63;
  const int t = lane & 3;
  const long long craw = (long long)vblock * Q::CPW + (lane >> 2);
  const bool active = t < N && craw < G.ncells;
  const int cell = (int)(craw < G.ncells ? craw : G.ncells - 1);
  const int ts = t < N ? t : N - 1;  // theta slice held by this lane
  const CellId C = decode_cell(G, cell);

  // every load that does not depend on arithmetic is issued here, before the
  // nodal values are used, so that their latencies overlap: the cos/sin of the
  // lane's theta point, the linearization data of the first point (then kept
  // one point ahead, points in (q, qj) order) and the nodal values
  Real trc, trs;
  {
    const Real* tr = G.trig + (((size_t)(C.dom ? G.nth[0] : 0) + C.ct) * N + ts) * 2;
    trc = tr[0];
    trs = tr[1];
  }
  constexpr int PF = 1;
  const Real* lbase = lin + ((size_t)cell * Q::NPT + ts) * LW;
  Real ring[PF][LW];
  if constexpr (!ULDS) {
#pragma unroll
    for (int i = 0; i < PF; ++i)
      if (i < Q::PL) load_lin<Real, LW>(lbase + ((i / N) * Q::PL + (i % N) * N) * LW, ring[i]);
  }

  // nodal values of the slice, constrained entries read as zero
  // ULDS: point values in LDS at us[((comp * N + r) * N + z) * 64 + lane]
  // (lane-owned columns, 4 N^2 values per lane)
  Real U[NC][N][N];  // [comp][r][z]
  Real SP[LINC ? DIM : 1][N][N];  // LINC: state velocity, nodal then point values
  {
    int it = k * C.ct + ts;
    const int ntn = pick(C.dom, G.ntd);
    it = it >= ntn ? it - ntn : it;
    const int nrn = pick(C.dom, G.nrn);
    const long long nbase = (C.dom ? G.node_off1 : 0) + it + (long long)ntn * (k * C.cr + (long long)nrn * k * C.cz);
#pragma unroll
    for (int b = 0; b < N; ++b)
#pragma unroll
      for (int c = 0; c < N; ++c) {
        const int ir = k * C.cr + b, iz = k * C.cz + c;
        const long long node = nbase + (long long)ntn * (b + (long long)nrn * c);
        Real w[4];
        load_node4<Real>(src + node * NC, w);
        if constexpr (LINC) {
          // the state enters with its boundary values (no constraint)
          Real ws[4];
          load_node4<Real>(state + node * NC, ws);
#pragma unroll
          for (int m = 0; m < DIM; ++m) SP[m][b][c] = ws[m];
        }
        const bool outer = (C.dom == 0) ? (ir == 0) : (ir == G.nrn[1] - 1);
        const bool vf = outer | (iz == 0) | (iz == G.nzn - 1);
        const bool pf = (C.dom == 1) & (it == 0) & (ir == G.nrn[1] - 1) & (iz == 0);
#pragma unroll
        for (int m = 0; m < DIM; ++m) U[m][b][c] = vf ? Real(0) : w[m];
        U[DIM][b][c] = pf ? Real(0) : w[DIM];
      }
  }

  // interpolation to the Gauss points: z, r in registers, theta across the quad
  {
    Real cV[N];
#pragma unroll
    for (int s = 0; s < N; ++s) {
      Real a[N];
#pragma unroll
      for (int i = 0; i < N; ++i) a[i] = T.V[i][(i + s) % N];
      cV[s] = lane_select<N>(ts, a);
    }
#pragma unroll
    for (int m = 0; m < NC; ++m) {
      Real A[N][N];
#pragma unroll
      for (int b = 0; b < N; ++b)
#pragma unroll
        for (int q = 0; q < N; ++q) {
          Real v = 0;
#pragma unroll
          for (int c = 0; c < N; ++c) v += T.V[q][c] * U[m][b][c];
          A[b][q] = v;
        }
#pragma unroll
      for (int qj = 0; qj < N; ++qj)
#pragma unroll
        for (int q = 0; q < N; ++q) {
          Real v = 0;
#pragma unroll
          for (int b = 0; b < N; ++b) v += T.V[qj][b] * A[b][q];
          Real xs[N];
          quad_rotate<N>(v, xs);
          const Real uq = quad_dot<N>(cV, xs);
          if constexpr (ULDS) us[((m * N + qj) * N + q) * 64 + lane] = uq;
          else U[m][qj][q] = uq;
        }
      __builtin_amdgcn_sched_barrier(0);
    }
    if constexpr (LINC) {
#pragma unroll
      for (int m = 0; m < DIM; ++m) {
        Real A[N][N];
#pragma unroll
        for (int b = 0; b < N; ++b)
#pragma unroll
          for (int q = 0; q < N; ++q) {
            Real v = 0;
#pragma unroll
            for (int c = 0; c < N; ++c) v += T.V[q][c] * SP[m][b][c];
            A[b][q] = v;
          }
#pragma unroll
        for (int qj = 0; qj < N; ++qj)
#pragma unroll
          for (int q = 0; q < N; ++q) {
            Real v = 0;
#pragma unroll
            for (int b = 0; b < N; ++b) v += T.V[qj][b] * A[b][q];
            Real xs[N];
            quad_rotate<N>(v, xs);
            const Real sq = quad_dot<N>(cV, xs);
            if constexpr (ULDS) ss[((m * N + qj) * N + q) * 64 + lane] = sq;
            else SP[m][qj][q] = sq;
          }
        __builtin_amdgcn_sched_barrier(0);
      }
    }
  }

  // per-lane theta coefficients of the collocation derivatives, applied to
  // the quad-rotated values (xs[s] from lane ts+s): rows cX[s] = X[ts][ts+s]
  // and, for the transposed contraction, columns tX[s] = X[ts+s][ts]
  // (indices mod N)
  Real cD[N], cDD[N], tD[N];
#pragma unroll
  for (int s = 0; s < N; ++s) {
    Real a[N], b[N], c[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
      a[i] = T.CD[i][(i + s) % N];
      b[i] = T.CDD[i][(i + s) % N];
      c[i] = T.CD[(i + s) % N][i];
    }
    cD[s] = lane_select<N>(ts, a);
    cDD[s] = lane_select<N>(ts, b);
    tD[s] = lane_select<N>(ts, c);
  }

  // geometry of the lane's theta point
  PtGeom<Real> g;
  g.c = trc;
  g.s = trs;
  const Real dr = pick(C.dom, G.dr), r0 = pick(C.dom, G.r0);
  g.inv_dr = Real(1) / dr;
  g.inv_dz = Real(1) / G.dz;
  const Real dth_c = pick(C.dom, G.dthd);
  const Real wt = lane_select<N>(ts, T.w) * dth_c * dr * G.dz;
  const Real nu = G.nu, ct = G.ct;
  const Real inv_dth = Real(1) / dth_c;
  Real rq[N], inv_rq[N];
#pragma unroll
  for (int qj = 0; qj < N; ++qj) {
    rq[qj] = r0 + dr * (Real(C.cr) + T.x[qj]);
    inv_rq[qj] = Real(1) / rq[qj];
  }

  Real F[NC][N][N];  // test coefficients in the collocation basis
#pragma unroll
  for (int m = 0; m < NC; ++m)
#pragma unroll
    for (int b = 0; b < N; ++b)
#pragma unroll
      for (int c = 0; c < N; ++c) F[m][b][c] = 0;

  Real lv[LL::SIZE];

#pragma unroll
  for (int q = 0; q < N; ++q)
#pragma unroll
    for (int qj = 0; qj < N; ++qj) {
      const int pt = q * N + qj;
      Real lw[LW];  // the point's stored values (all 16, or tau and tau R)
      if constexpr (ULDS) {
        load_lin<Real, LW>(lbase + ((pt / N) * Q::PL + (pt % N) * N) * LW, lw);
      } else {
#pragma unroll
        for (int j = 0; j < LW; ++j) lw[j] = ring[0][j];
#pragma unroll
        for (int i = 0; i + 1 < PF; ++i)
#pragma unroll
          for (int j = 0; j < LW; ++j) ring[i][j] = ring[i + 1][j];
        if (pt + PF < Q::PL)
          load_lin<Real, LW>(lbase + (((pt + PF) / N) * Q::PL + ((pt + PF) % N) * N) * LW, ring[PF - 1]);
      }
      if constexpr (!LINC) {
#pragma unroll
        for (int j = 0; j < LL::SIZE; ++j) lv[j] = lw[j];
      } else {
        lv[LL::TAU] = lw[0];
#pragma unroll
        for (int m = 0; m < DIM; ++m) lv[LL::TR + m] = lw[1 + m];
      }
      RefVal<Real, DIM> rv[DIM], rp;
#pragma unroll
      for (int m = 0; m < NC; ++m) {
        const bool vel = m < DIM;
        RefVal<Real, DIM>& R = vel ? rv[m] : rp;
        // point values of this component along r (at q) and z (at qj)
        Real ur[N], uz[N];
#pragma unroll
        for (int j = 0; j < N; ++j) {
          if constexpr (ULDS) {
            ur[j] = us[((m * N + j) * N + q) * 64 + lane];
            uz[j] = us[((m * N + qj) * N + j) * 64 + lane];
          } else {
            ur[j] = U[m][j][q];
            uz[j] = U[m][qj][j];
          }
        }
        const Real v = ur[qj];
        Real d1 = T.CD[qj][0] * ur[0], e1 = T.CD[q][0] * uz[0];
        Real d2 = vel ? T.CDD[qj][0] * ur[0] : Real(0), e2 = vel ? T.CDD[q][0] * uz[0] : Real(0);
#pragma unroll
        for (int j = 1; j < N; ++j) {
          d1 += T.CD[qj][j] * ur[j];
          e1 += T.CD[q][j] * uz[j];
          if (vel) {
            d2 += T.CDD[qj][j] * ur[j];
            e2 += T.CDD[q][j] * uz[j];
          }
        }
        Real xs[N];
        quad_rotate<N>(v, xs);
        R.v = v;
        R.d[0] = quad_dot<N>(cD, xs);
        R.d[1] = d1;
        R.d[2] = e1;
        R.dd[0] = vel ? quad_dot<N>(cDD, xs) : Real(0);
        R.dd[1] = d2;
        R.dd[2] = e2;
      }
      g.r = rq[qj];
      g.inv_r = inv_rq[qj];
      g.inv_rdth = g.inv_r * inv_dth;
      g.jxw = wt * T.w[qj] * T.w[q] * g.r;
      g.complete();
      if constexpr (LINC) {
        // mesh velocity omega e_z x x in rotor cells
        const Real w0 = C.dom == 0 ? -G.omega * g.r * g.s : Real(0);
        const Real w1 = C.dom == 0 ? G.omega * g.r * g.c : Real(0);
#pragma unroll
        for (int m = 0; m < DIM; ++m) {
          Real sr[N], sz[N];
#pragma unroll
          for (int j = 0; j < N; ++j) {
            if constexpr (ULDS) {
              sr[j] = ss[((m * N + j) * N + q) * 64 + lane];
              sz[j] = ss[((m * N + qj) * N + j) * 64 + lane];
            } else {
              sr[j] = SP[m][j][q];
              sz[j] = SP[m][qj][j];
            }
          }
          const Real v = sr[qj];
          Real d1 = T.CD[qj][0] * sr[0], e1 = T.CD[q][0] * sz[0];
#pragma unroll
          for (int j = 1; j < N; ++j) {
            d1 += T.CD[qj][j] * sr[j];
            e1 += T.CD[q][j] * sz[j];
          }
          Real xs[N];
          quad_rotate<N>(v, xs);
          const Real d0 = quad_dot<N>(cD, xs);
          lv[LL::A + m] = v - (m == 0 ? w0 : m == 1 ? w1 : Real(0));
          // reference derivatives (theta d0, r d1, z e1) -> Cartesian gradient
          const Real gx = g.a1 * d1 - g.b2 * d0, gy = g.a2 * d1 + g.b1 * d0, gz = e1 * g.inv_dz;
          lv[LL::GU + m * DIM + 0] = picard ? Real(0) : gx;
          lv[LL::GU + m * DIM + 1] = picard ? Real(0) : gy;
          lv[LL::GU + m * DIM + 2] = picard ? Real(0) : gz;
        }
      }
      Real tc[NC][NT];
      pointwise_jacobian<Real, DIM>(g, rv, rp, lv, nu, ct, tc);
#pragma unroll
      for (int m = 0; m < NC; ++m) {
        Real xs[N];
        quad_rotate<N>(tc[m][1], xs);
        Real f = F[m][qj][q] + tc[m][0];
#pragma unroll
        for (int s = 0; s < N; ++s) f += tD[s] * xs[s];
        F[m][qj][q] = f;
#pragma unroll
        for (int j = 0; j < N; ++j) {
          F[m][j][q] += T.CD[qj][j] * tc[m][2];
          F[m][qj][j] += T.CD[q][j] * tc[m][3];
        }
      }
      // pin the accumulators at the end of every point (otherwise the
      // additions are deferred and every product stays live), and keep the
      // scheduler from interleaving points
#pragma unroll
      for (int m = 0; m < NC; ++m)
#pragma unroll
        for (int b = 0; b < N; ++b)
#pragma unroll
          for (int c = 0; c < N; ++c) asm volatile("" : "+v"(F[m][b][c]));
      __builtin_amdgcn_sched_barrier(0);
    }

  // back to the nodes: transposed interpolation across the quad (theta),
  // then along r and z in registers
  Real tV[N];
#pragma unroll
  for (int s = 0; s < N; ++s) {
    Real a[N];
#pragma unroll
    for (int i = 0; i < N; ++i) a[i] = T.V[(i + s) % N][i];
    tV[s] = lane_select<N>(ts, a);
  }
  Real* Ec = E + cell;
  // strip layout: the 16 cells of the wavefront are theta-consecutive, so the
  // theta-face shared by cells i-1 and i is summed here and the batch stores
  // 16 k + 1 node columns per (r, z) node position instead of 16 (k + 1).
  // Lane (i, 0) adds the value of the lane just before it, lane (i-1, 3),
  // which holds slice k of cell i-1 (for k = 2 it duplicates lane (i-1, 2)).
  // Columns 0 .. 16k-1 of a batch are contiguous (aligned 16 k values per
  // batch and node position); column 16k, the face shared with the next
  // batch, goes to a separate array after them.
  constexpr int KD = N - 1, SL = 16 * KD;
  const int ci = lane >> 2;
  const bool store_s = active && (ts < KD || ci == Q::CPW - 1);
  const size_t nblk = (size_t)(G.ncells / Q::CPW);
  const size_t pstride = nblk * SL;  // per (comp, z, r) node position
  Real* Es = (ts < KD) ? E + (size_t)vblock * SL + KD * ci + ts : E + (size_t)N * N * NC * pstride + vblock;
  const size_t estride = (ts < KD) ? pstride : nblk;
#pragma unroll
  for (int m = 0; m < NC; ++m) {
    Real X[N][N];
#pragma unroll
    for (int qj = 0; qj < N; ++qj)
#pragma unroll
      for (int q = 0; q < N; ++q) {
        Real xs[N];
        quad_rotate<N>(F[m][qj][q], xs);
        X[qj][q] = quad_dot<N>(tV, xs);
      }
    Real Y[N][N];
#pragma unroll
    for (int b = 0; b < N; ++b)
#pragma unroll
      for (int q = 0; q < N; ++q) {
        Real v = 0;
#pragma unroll
        for (int qj = 0; qj < N; ++qj) v += T.V[qj][b] * X[qj][q];
        Y[b][q] = v;
      }
#pragma unroll
    for (int b = 0; b < N; ++b)
#pragma unroll
      for (int c = 0; c < N; ++c) {
        Real v = 0;
#pragma unroll
        for (int q = 0; q < N; ++q) v += T.V[q][c] * Y[b][q];
        if (strip) {
          const Real nb = from_prev_lane(v);
          if (t == 0 && ci > 0) v += nb;
          if (store_s) Es[(size_t)((m * N + c) * N + b) * estride] = v;
        } else if (active) {
          Ec[(size_t)(m * Q::NPT + c * Q::PL + b * N + ts) * G.ncells] = v;
        }
      }
    __builtin_amdgcn_sched_barrier(0);
  }
}

template <typename Real, int N, bool LINC = false>
__global__ __launch_bounds__(64) void k_jacobian_volume_quad(Geom<Real> G, Tab1D<Real, N> T, int k,
                                                             const Real* __restrict__ lin,
                                                             const Real* __restrict__ src, Real* __restrict__ E,
                                                             int strip, const Real* __restrict__ state,
                                                             int picard) {
  constexpr bool kLds = sizeof(Real) == 8;
  __shared__ Real us[kLds ? (LINC ? 7 : 4) * N * N * 64 : 1];
  volume_quad<Real, N, kLds, LINC>(G, T, k, blockIdx.x, lin, src, E, strip != 0, us, state, picard);
}

// ---------------------------------------------------------------------------
// State kernel: per-point linearization data (LIN) or nonlinear residual (RES)
// ---------------------------------------------------------------------------
template <int DIM, int N, bool RES>
__global__ __launch_bounds__(64) void k_state(Geom<double> G, Tab1D<double, N> T, int k,
                                              const double* __restrict__ state, const double* __restrict__ hist,
                                              const double* __restrict__ force, double* __restrict__ lin,
                                              double* __restrict__ res, int picard) {
  using Real = double;
  using S = Shape<Real, DIM, N>;
  using LL = LinLayout<DIM>;
  constexpr int NZ = S::NZ, NC = S::NC;
  constexpr int XSLOT = S::EVAL_SLOTS;  // first slot of the value-only fields
  constexpr int SL = (S::SLOTS > XSLOT + 2 * DIM) ? S::SLOTS : XSLOT + 2 * DIM;
  __shared__ Real lds[S::template lds_size<SL>()];
  __shared__ Tab1D<Real, N> sT;
  const int lane = threadIdx.x;
  {
    constexpr int NW = (int)(sizeof(Tab1D<Real, N>) / sizeof(Real));
    const Real* tw = (const Real*)&T;
    for (int i = lane; i < NW; i += 64) ((Real*)&sT)[i] = tw[i];
  }
  const int cl = lane / S::TPC;
  const int t = lane % S::TPC;
  const int ta = t % N, tb = t / N;
  const int cell = blockIdx.x * S::CPW + cl;
  const bool active = cl < S::CPW && cell < G.ncells;
  Real* L = lds + (active ? cl : 0) * (SL * S::NPT);
  CellId C = decode_cell(G, active ? cell : 0);
  const bool has_hist = hist != nullptr, has_force = force != nullptr;

  Real u[NC][NZ];
  if (active) gather_line<Real, DIM, N>(G, k, C, ta, tb, state, false, u);
  eval_stage_z<Real, DIM, N, DIM, true>(T, u, L, ta, tb, active);
  // value-only fields: history and force, reduced along z and r right here
  if (active && (has_hist || has_force)) {
    for (int f = 0; f < 2; ++f) {
      const double* v = f == 0 ? hist : force;
      if (!v) continue;
      Real w[NC][NZ];
      gather_line<Real, DIM, N>(G, k, C, ta, tb, v, false, w);
#pragma unroll
      for (int m = 0; m < DIM; ++m) {
#pragma unroll
        for (int q = 0; q < NZ; ++q) {
          Real s = 0;
          if constexpr (DIM == 3) {
#pragma unroll
            for (int c = 0; c < NZ; ++c) s += T.V[q][c] * w[m][c];
          } else {
            s = w[m][0];
          }
          L[((XSLOT + f * DIM + m) * S::NPT + q * S::PLANE + tb * N + ta) * S::ES] = s;
        }
      }
    }
  }
  __syncthreads();
  if (has_hist || has_force) {
    Real o[2 * DIM][NZ];
    if (active) {
      for (int f = 0; f < 2 * DIM; ++f)
#pragma unroll
        for (int q = 0; q < NZ; ++q) {
          Real s = 0;
#pragma unroll
          for (int b = 0; b < N; ++b) s += sT.V[tb][b] * L[((XSLOT + f) * S::NPT + q * S::PLANE + b * N + ta) * S::ES];
          o[f][q] = s;
        }
    }
    __syncthreads();
    if (active)
      for (int f = 0; f < 2 * DIM; ++f)
#pragma unroll
        for (int q = 0; q < NZ; ++q) L[((XSLOT + f) * S::NPT + q * S::PLANE + tb * N + ta) * S::ES] = o[f][q];
  }
  eval_stage_r<Real, DIM, N, DIM, true>(sT, L, ta, tb, active);

  Real tc[NZ][NC][S::NT];
  if (active) {
    const Real nu = G.nu, ct = G.ct;
    const Real hc = G.hcell[C.dom * G.hstride + C.cr];
    const Real ih2 = 1.0 / (hc * hc);
    const Real visc = 9.0 * (4.0 * nu * ih2) * (4.0 * nu * ih2);
#pragma unroll
    for (int q = 0; q < NZ; ++q) {
      RefVal<Real, DIM> rv[DIM], rp;
#pragma unroll
      for (int m = 0; m < DIM; ++m) eval_stage_t_vel<Real, DIM, N>(sT, L, m * S::NYV, ta, tb, q, rv[m]);
      eval_stage_t_pres<Real, DIM, N>(sT, L, DIM * S::NYV, ta, tb, q, rp);
      const PtGeom<Real> g = point_geom<Real, DIM, N>(G, sT, C, ta, tb, q);
      Real uu[DIM], gu[DIM][DIM], lu[DIM], gp[DIM], dummy, hv[DIM], fv[DIM];
#pragma unroll
      for (int m = 0; m < DIM; ++m) {
        uu[m] = rv[m].v;
        to_physical<Real, DIM>(g, nullptr, rv[m], gu[m], lu[m], true);
        hv[m] = (has_hist && ct != 0) ? eval_stage_t_value<Real, DIM, N>(sT, L, XSLOT + m, ta, tb, q) : 0.0;
        fv[m] = has_force ? eval_stage_t_value<Real, DIM, N>(sT, L, XSLOT + DIM + m, ta, tb, q) : 0.0;
      }
      to_physical<Real, DIM>(g, nullptr, rp, gp, dummy, false);
      // mesh velocity omega e_z x x in rotor cells
      Real w[DIM] = {};
      if (C.dom == 0) {
        w[0] = -G.omega * g.r * g.s;
        w[1] = G.omega * g.r * g.c;
      }
      Real a[DIM], an2 = 0;
#pragma unroll
      for (int m = 0; m < DIM; ++m) {
        a[m] = uu[m] - w[m];
        an2 += a[m] * a[m];
      }
      const Real tau = 1.0 / sqrt(G.ctau2 + 4.0 * an2 * ih2 + visc);
      Real R[DIM], conv[DIM];
#pragma unroll
      for (int m = 0; m < DIM; ++m) {
        Real s = 0;
#pragma unroll
        for (int e = 0; e < DIM; ++e) s += gu[m][e] * a[e];
        conv[m] = s;
        R[m] = ct * uu[m] + hv[m] + s + gp[m] - nu * lu[m] - fv[m];
      }
      if constexpr (!RES) {
        double* lp = lin + ((size_t)cell * S::NPT + q * S::PLANE + tb * N + ta) * LL::SIZE;
#pragma unroll
        for (int m = 0; m < DIM; ++m) {
          // Picard (Oseen) linearization: no reaction term (zero velocity
          // gradient) and no SUPG weight derivative (zero tau R)
          lp[LL::A + m] = a[m];
          lp[LL::TR + m] = picard ? 0.0 : tau * R[m];
#pragma unroll
          for (int e = 0; e < DIM; ++e) lp[LL::GU + m * DIM + e] = picard ? 0.0 : gu[m][e];
        }
        lp[LL::TAU] = tau;
      } else {
        Real divu = 0;
#pragma unroll
        for (int m = 0; m < DIM; ++m) {
          divu += gu[m][m];
          Real Gm[DIM];
#pragma unroll
          for (int e = 0; e < DIM; ++e) Gm[e] = nu * gu[m][e] + tau * R[m] * a[e];
          Gm[m] -= rp.v;
          to_reference<Real, DIM>(g, ct * uu[m] + hv[m] + conv[m] - fv[m], Gm, tc[q][m]);
        }
        Real Gq[DIM];
#pragma unroll
        for (int e = 0; e < DIM; ++e) Gq[e] = tau * R[e];
        to_reference<Real, DIM>(g, divu, Gq, tc[q][DIM]);
      }
    }
  }
  if constexpr (RES) {
    __syncthreads();
    if (active) {
#pragma unroll
      for (int q = 0; q < NZ; ++q)
#pragma unroll
        for (int m = 0; m < NC; ++m)
#pragma unroll
          for (int j = 0; j < S::NT; ++j) L[((m * S::NT + j) * S::NPT + q * S::PLANE + tb * N + ta) * S::ES] = tc[q][m][j];
    }
    __syncthreads();
    integrate_store<Real, DIM, N>(sT, T, L, ta, tb, active, cell, G.ncells, res);
  }
}

// ---------------------------------------------------------------------------
// State kernel on iso-parametric cells: the same outputs as k_state.  The
// cell's nodal state (and history, force) is staged in LDS and every point is
// evaluated directly from the tensor basis, mixed second derivatives
// included; the metric comes from the per-point table (G.geo), the mesh
// velocity from the point positions (G.geox), tau from the cell's h (G.hiso).
// Not on the Jacobian's hot path: it runs once per linearization.
// ---------------------------------------------------------------------------
template <int DIM, int N, bool RES>
__global__ __launch_bounds__(64) void k_state_iso(Geom<double> G, Tab1D<double, N> T, int k,
                                                  const double* __restrict__ state, const double* __restrict__ hist,
                                                  const double* __restrict__ force, double* __restrict__ lin,
                                                  double* __restrict__ res, int picard) {
  using Real = double;
  using S = Shape<Real, DIM, N>;
  using LL = LinLayout<DIM>;
  constexpr int NZ = S::NZ, NC = S::NC, NPT = S::NPT, NU = NC + 2 * DIM;
  __shared__ Real U[S::CPW][NU][NPT];                   // state, history, force at the cell's nodes
  __shared__ Real L[S::CPW * S::TEST_SLOTS * NPT];       // test coefficients (residual)
  __shared__ Tab1D<Real, N> sT;
  const int lane = threadIdx.x;
  {
    constexpr int NW = (int)(sizeof(Tab1D<Real, N>) / sizeof(Real));
    const Real* tw = (const Real*)&T;
    for (int i = lane; i < NW; i += 64) ((Real*)&sT)[i] = tw[i];
  }
  const int cl = lane / S::TPC;
  const int t = lane % S::TPC;
  const int ta = t % N, tb = t / N;
  const int cell = blockIdx.x * S::CPW + cl;
  const bool active = cl < S::CPW && cell < G.ncells;
  const CellId C = decode_cell(G, active ? cell : 0);
  const bool has_hist = hist != nullptr, has_force = force != nullptr;
  if (active) {
    for (int node = t; node < NPT; node += S::TPC) {
      const int a = node % N, b = (node / N) % N, c = node / S::PLANE;
      int it, ir, iz;
      const long long nd = node_of<Real, DIM>(G, k, C, a, b, c, it, ir, iz);
#pragma unroll
      for (int m = 0; m < NC; ++m) U[cl][m][node] = state[nd * NC + m];
#pragma unroll
      for (int m = 0; m < DIM; ++m) {
        U[cl][NC + m][node] = has_hist ? hist[nd * NC + m] : 0.0;
        U[cl][NC + DIM + m][node] = has_force ? force[nd * NC + m] : 0.0;
      }
    }
  }
  __syncthreads();
  Real* Lc = L + (active ? cl : 0) * (S::TEST_SLOTS * NPT);
  if (active) {
    const Real nu = G.nu, ct = G.ct;
    const Real hc = G.hiso[cell];
    const Real ih2 = 1.0 / (hc * hc);
    const Real visc = 9.0 * (4.0 * nu * ih2) * (4.0 * nu * ih2);
    for (int q = 0; q < NZ; ++q) {
      const int pt = q * S::PLANE + tb * N + ta;
      // values, reference gradients and Hessians of the velocity; values and
      // gradients of the pressure; values of history and force
      Real uv[DIM], ud[DIM][DIM], udd[DIM][DIM], umx[DIM][3], pv = 0, pd[DIM], hv[DIM], fv[DIM];
#pragma unroll
      for (int m = 0; m < DIM; ++m) {
        uv[m] = hv[m] = fv[m] = 0;
#pragma unroll
        for (int e = 0; e < DIM; ++e) ud[m][e] = udd[m][e] = 0;
        umx[m][0] = umx[m][1] = umx[m][2] = 0;
        pd[m] = 0;
      }
      for (int c = 0; c < NZ; ++c) {
        const Real z0 = DIM == 3 ? sT.V[q][c] : 1.0, z1 = DIM == 3 ? sT.D[q][c] : 0.0,
                   z2 = DIM == 3 ? sT.DD[q][c] : 0.0;
        for (int b = 0; b < N; ++b) {
          const Real r0 = sT.V[tb][b], r1 = sT.D[tb][b], r2 = sT.DD[tb][b];
#pragma unroll
          for (int a = 0; a < N; ++a) {
            const Real t0 = sT.V[ta][a], t1 = sT.D[ta][a], t2 = sT.DD[ta][a];
            const int node = (c * N + b) * N + a;
            const Real phi = t0 * r0 * z0;
            const Real dphi[3] = {t1 * r0 * z0, t0 * r1 * z0, t0 * r0 * z1};
            const Real ddphi[3] = {t2 * r0 * z0, t0 * r2 * z0, t0 * r0 * z2};
            const Real mxphi[3] = {t1 * r1 * z0, t1 * r0 * z1, t0 * r1 * z1};
#pragma unroll
            for (int m = 0; m < DIM; ++m) {
              const Real u = U[cl][m][node];
              uv[m] += phi * u;
#pragma unroll
              for (int e = 0; e < DIM; ++e) {
                ud[m][e] += dphi[e] * u;
                udd[m][e] += ddphi[e] * u;
              }
#pragma unroll
              for (int e = 0; e < 3; ++e) umx[m][e] += mxphi[e] * u;
              hv[m] += phi * U[cl][NC + m][node];
              fv[m] += phi * U[cl][NC + DIM + m][node];
            }
            const Real p = U[cl][DIM][node];
            pv += phi * p;
#pragma unroll
            for (int e = 0; e < DIM; ++e) pd[e] += dphi[e] * p;
          }
        }
      }
      IsoPt<Real, DIM> g;
      g.load(G.geo + ((size_t)cell * NPT + pt) * IsoLayout<DIM>::SIZE);
      Real gu[DIM][DIM], lu[DIM], gp[DIM], dummy;
#pragma unroll
      for (int m = 0; m < DIM; ++m) {
        RefValX<Real, DIM> rv;
        rv.v = uv[m];
#pragma unroll
        for (int e = 0; e < DIM; ++e) {
          rv.d[e] = ud[m][e];
          rv.dd[e] = udd[m][e];
        }
        rv.mx[0] = umx[m][0];
        rv.mx[1] = umx[m][1];
        rv.mx[2] = umx[m][2];
        to_physical<Real, DIM>(g, nullptr, rv, gu[m], lu[m], true);
        if (!(has_hist && ct != 0)) hv[m] = 0;
      }
      {
        RefValX<Real, DIM> rp;
        rp.v = pv;
#pragma unroll
        for (int e = 0; e < DIM; ++e) {
          rp.d[e] = pd[e];
          rp.dd[e] = 0;
        }
        rp.mx[0] = rp.mx[1] = rp.mx[2] = 0;
        to_physical<Real, DIM>(g, nullptr, rp, gp, dummy, false);
      }
      // mesh velocity omega e_z x x in rotor cells
      const double* xp = G.geox + ((size_t)cell * NPT + pt) * 3;
      Real w[DIM] = {};
      if (C.dom == 0) {
        w[0] = -G.omega * xp[1];
        w[1] = G.omega * xp[0];
      }
      Real a[DIM], an2 = 0;
#pragma unroll
      for (int m = 0; m < DIM; ++m) {
        a[m] = uv[m] - w[m];
        an2 += a[m] * a[m];
      }
      const Real tau = 1.0 / sqrt(G.ctau2 + 4.0 * an2 * ih2 + visc);
      Real R[DIM], conv[DIM];
#pragma unroll
      for (int m = 0; m < DIM; ++m) {
        Real s2 = 0;
#pragma unroll
        for (int e = 0; e < DIM; ++e) s2 += gu[m][e] * a[e];
        conv[m] = s2;
        R[m] = ct * uv[m] + hv[m] + s2 + gp[m] - nu * lu[m] - fv[m];
      }
      if constexpr (!RES) {
        double* lp = lin + ((size_t)cell * NPT + pt) * LL::SIZE;
#pragma unroll
        for (int m = 0; m < DIM; ++m) {
          lp[LL::A + m] = a[m];
          lp[LL::TR + m] = picard ? 0.0 : tau * R[m];
#pragma unroll
          for (int e = 0; e < DIM; ++e) lp[LL::GU + m * DIM + e] = picard ? 0.0 : gu[m][e];
        }
        lp[LL::TAU] = tau;
      } else {
        Real tc[NC][S::NT];
        Real divu = 0;
#pragma unroll
        for (int m = 0; m < DIM; ++m) {
          divu += gu[m][m];
          Real Gm[DIM];
#pragma unroll
          for (int e = 0; e < DIM; ++e) Gm[e] = nu * gu[m][e] + tau * R[m] * a[e];
          Gm[m] -= pv;
          to_reference<Real, DIM>(g, ct * uv[m] + hv[m] + conv[m] - fv[m], Gm, tc[m]);
        }
        Real Gq[DIM];
#pragma unroll
        for (int e = 0; e < DIM; ++e) Gq[e] = tau * R[e];
        to_reference<Real, DIM>(g, divu, Gq, tc[DIM]);
#pragma unroll
        for (int m = 0; m < NC; ++m)
#pragma unroll
          for (int j = 0; j < S::NT; ++j) Lc[(m * S::NT + j) * NPT + pt] = tc[m][j];
      }
    }
  }
  if constexpr (RES) {
    __syncthreads();
    integrate_store<Real, DIM, N>(sT, T, Lc, ta, tb, active, cell, G.ncells, res);
  }
}

// ---------------------------------------------------------------------------
// Volume diagonal (column i of the element matrix, entry i) from stored
// linearization data: one lane per (cell, local DoF), loop over points.
// ---------------------------------------------------------------------------
template <typename Real, int DIM, int N, bool ISO = false>
__global__ __launch_bounds__(128) void k_diag_volume(Geom<Real> G, Tab1D<Real, N> T, int k,
                                                     const Real* __restrict__ lin, Real* __restrict__ diag) {
  // one thread per (cell, node): the basis function, its physical derivatives
  // and the point data are shared by the node's d + 1 components
  using S = Shape<Real, DIM, N>;
  using LL = LinLayout<DIM>;
  constexpr int NZ = S::NZ, NC = S::NC;
  const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long total = (long long)G.ncells * S::NPT;
  if (gid >= total) return;
  const int node = gid % S::NPT;
  const int cell = gid / S::NPT;
  const int a0 = node % N, a1 = (node / N) % N, a2 = node / S::PLANE;
  const CellId C = decode_cell(G, cell);
  const Real nu = G.nu, ct = G.ct;
  Real acc[NC];
#pragma unroll
  for (int m = 0; m < NC; ++m) acc[m] = 0;
  for (int q = 0; q < NZ; ++q)
    for (int qj = 0; qj < N; ++qj)
      for (int qi = 0; qi < N; ++qi) {
        const Real vz = (DIM == 3) ? T.V[q][a2] : Real(1);
        const Real dz_ = (DIM == 3) ? T.D[q][a2] : Real(0);
        const Real ddz = (DIM == 3) ? T.DD[q][a2] : Real(0);
        using RV = std::conditional_t<ISO, RefValX<Real, DIM>, RefVal<Real, DIM>>;
        RV rv;
        rv.v = T.V[qi][a0] * T.V[qj][a1] * vz;
        rv.d[0] = T.D[qi][a0] * T.V[qj][a1] * vz;
        rv.d[1] = T.V[qi][a0] * T.D[qj][a1] * vz;
        rv.dd[0] = T.DD[qi][a0] * T.V[qj][a1] * vz;
        rv.dd[1] = T.V[qi][a0] * T.DD[qj][a1] * vz;
        if constexpr (DIM == 3) {
          rv.d[2] = T.V[qi][a0] * T.V[qj][a1] * dz_;
          rv.dd[2] = T.V[qi][a0] * T.V[qj][a1] * ddz;
        }
        Real gphi[DIM], lphi, jxw;
        if constexpr (ISO) {
          rv.mx[0] = T.D[qi][a0] * T.D[qj][a1] * vz;
          rv.mx[1] = T.D[qi][a0] * T.V[qj][a1] * dz_;
          rv.mx[2] = T.V[qi][a0] * T.D[qj][a1] * dz_;
          IsoPt<Real, DIM> g;
          g.load(G.geo + ((size_t)cell * S::NPT + q * S::PLANE + qj * N + qi) * IsoLayout<DIM>::SIZE);
          to_physical<Real, DIM>(g, nullptr, rv, gphi, lphi, true);
          jxw = g.jxw;
        } else {
          const PtGeom<Real> g = point_geom<Real, DIM, N>(G, T, C, qi, qj, q);
          to_physical<Real, DIM>(g, nullptr, rv, gphi, lphi, true);
          jxw = g.jxw;
        }
        const Real phi = rv.v;
        const Real* lp = lin + ((size_t)cell * S::NPT + q * S::PLANE + qj * N + qi) * LL::SIZE;
        const Real tau = lp[LL::TAU];
        Real adg = 0, g2 = 0;
#pragma unroll
        for (int e = 0; e < DIM; ++e) {
          adg += lp[LL::A + e] * gphi[e];
          g2 += gphi[e] * gphi[e];
        }
#pragma unroll
        for (int comp = 0; comp < DIM; ++comp) {
          // trial phi e_c tested with phi e_c (Sec. 2.3, A-hat diagonal)
          const Real guc = lp[LL::GU + comp * DIM + comp];
          const Real Rpc = (ct + guc) * phi + adg - nu * lphi;
          acc[comp] += jxw * (phi * phi * (ct + guc) + phi * adg + nu * g2 + tau * Rpc * adg +
                              lp[LL::TR + comp] * phi * gphi[comp]);
        }
        // D-hat diagonal: tau |grad psi|^2
        acc[DIM] += jxw * tau * g2;
      }
  int it, ir, iz;
  const long long nd = node_of<Real, DIM>(G, k, C, a0, a1, a2, it, ir, iz);
#pragma unroll
  for (int m = 0; m < NC; ++m) atomic_add(diag + nd * NC + m, acc[m]);
}

// ---------------------------------------------------------------------------
// Mortar face terms (Sec. 2.1, Eqs. EqMortarPre / EqMortarDiff / EqMortarMass
// with the mapped segment quadrature of Sec. 3.2).  One wavefront per
// interface cell side: it evaluates its own cell and the two cells of the
// other side that overlap it, forms the side's face coefficients at every
// mortar point and integrates them against its own test functions.
// ---------------------------------------------------------------------------
template <typename Real, int DIM, int N>
struct Piece {
  int seg;         // segment index (0 or 1) of the stator face
  int jface;       // stator face index (for the mortar point angles)
  CellId other;
};

template <typename Real, int DIM, int N>
__device__ inline void mortar_pieces(const Geom<Real>& G, int mstep, int side, int ct, int cz,
                                     Piece<Real, DIM, N> (&p)[2]) {
  const int nt = G.nth[0];  // equal counts on both sides
  if (side == 1) {
    const int j = ct;
    p[0].seg = 0;
    p[0].jface = j;
    p[1].seg = 1;
    p[1].jface = j;
    p[0].other = CellId{0, ((j - mstep - 1) % nt + nt) % nt, G.nr[0] - 1, cz};
    p[1].other = CellId{0, ((j - mstep) % nt + nt) % nt, G.nr[0] - 1, cz};
  } else {
    const int i = ct;
    const int j0 = (mstep + i) % nt, j1 = (mstep + i + 1) % nt;
    p[0].seg = 1;
    p[0].jface = j0;
    p[1].seg = 0;
    p[1].jface = j1;
    p[0].other = CellId{1, j0, 0, cz};
    p[1].other = CellId{1, j1, 0, cz};
  }
}

// Mortar kernel (Sec. 2.1 face terms with the mapped segment quadrature of
// Sec. 3.2).  A 64-lane block handles FPB interface cell sides ("faces"); each
// face couples its own cell with the two overlapping cells of the other side.
//   Phase A, lane = (face, piece, side, component): the lane loads the 27 (or
//     n^d) nodal values of that component of that cell and evaluates value and
//     reference derivatives at the piece's mortar points by sum factorization
//     in registers: r first (interface value and normal derivative), then
//     theta at the segment's points, then z at the Gauss points.
//   Phase B, lane = (face, piece, point): the own side's face coefficients
//     (jump = own - other, n = own outward normal).
//   Phase C, lane = (face, component, radial node row): the transposed sum
//     factorization integrates the coefficients against the own cell's test
//     functions; the result is stored as Em[comp][local node][face].
template <typename Real, int DIM, int N, int BUDGET = 36000>
struct MortarShape {
  static constexpr int NZ = (DIM == 3) ? N : 1;
  static constexpr int NC = DIM + 1;
  static constexpr int NQ = N * NZ;   // mortar points per piece
  static constexpr int NE = DIM + 1;  // value + reference derivatives
  static constexpr int LPF = 4 * NC;  // lanes per face in phase A
  // LDS row of one mortar point, padded by one value against bank conflicts
  // (every degree; rows hold NC * NE <= 16 values, so index NC * NE - 1 is
  // the last one a lane writes or reads)
  static constexpr int PQ = NC * NE + 1;
  static constexpr int PER_FACE = (2 * 2 * NQ * PQ + 2 * NQ * PQ) * (int)sizeof(Real);
  static constexpr int FPB0 = 64 / LPF;
  static constexpr int FPB_LDS = BUDGET / PER_FACE > 0 ? BUDGET / PER_FACE : 1;
  static constexpr int FPB = FPB0 < FPB_LDS ? FPB0 : FPB_LDS;
};

template <typename Real, int DIM, int N, int BUDGET = 36000>
struct MortarSmem {
  using MS = MortarShape<Real, DIM, N, BUDGET>;
  MortarTab<Real, N> M;
  Real trg[MS::FPB][2][N][2];
  // [face][piece][own=0 / other=1][point][comp * NE + quantity]; each point's
  // row is padded by one value so that lanes on consecutive points fall in
  // different LDS banks
  Real ev[MS::FPB][2][2][MS::NQ][MS::PQ];
  Real coef[MS::FPB][2][MS::NQ][MS::PQ];
};

// ISO: iso-parametric cells; phase B takes the inverse Jacobians of both
// sides at every point from iso_mg (IsoMortarLayout per face side, piece and
// point at the current angle) instead of the polar formulas
template <typename Real, int DIM, int N, int BUDGET = 36000, bool ISO = false>
__device__ inline void mortar_block(const Geom<Real>& G, const Tab1D<Real, N>& T, int k, int mblock,
                                    const MortarTab<Real, N>* __restrict__ Mp, const Real* __restrict__ mtrig,
                                    const Real* __restrict__ src, Real* __restrict__ Em, int mask,
                                    MortarSmem<Real, DIM, N, BUDGET>& sm, const Real* __restrict__ iso_mg = nullptr) {
  using S = Shape<Real, DIM, N>;
  using MS = MortarShape<Real, DIM, N, BUDGET>;
  constexpr int NC = MS::NC, NZ = MS::NZ, NQ = MS::NQ, NE = MS::NE, FPB = MS::FPB;
  MortarTab<Real, N>& M = sm.M;
  auto& trg = sm.trg;
  auto& ev = sm.ev;
  auto& coef = sm.coef;
  const int nfaces = G.nth[0] * G.nz;  // equal counts on both sides
  const int nsides = 2 * nfaces;
  // ---- phase A: evaluation.  Lane = (face, piece, side, component).  The
  // table copy's loads go first; the pairing of faces needs only the offset
  // m (read from the table in global memory), so the point angles and, when
  // they fit in registers, the lane's nodal values are loaded next, all
  // before the first wait.  Lanes past the last face read a valid face and
  // store nothing.
  constexpr bool EARLY = NZ * N * N <= 32;
  const int* srcw = (const int*)Mp;
  constexpr int NW = (int)(sizeof(MortarTab<Real, N>) / sizeof(int));
  constexpr int IT = (NW + 63) / 64;
  int w[IT];
#pragma unroll
  for (int j = 0; j < IT; ++j) {
    const int i = (int)threadIdx.x + 64 * j;
    w[j] = i < NW ? srcw[i] : 0;
  }
  const int fl = threadIdx.x / MS::LPF;
  const int lr = threadIdx.x % MS::LPF;
  const int m = lr % NC, sd = (lr / NC) % 2, pc = lr / (2 * NC);
  const int fs0 = mblock * FPB + fl;  // face-side index: side * nfaces + face
  const bool act = fl < FPB && fs0 < nsides;
  const int fs = act ? fs0 : nsides - 1;
  const int side = fs / nfaces, f = fs % nfaces;
  const int ct = f % G.nth[0], cz = f / G.nth[0];
  Piece<Real, DIM, N> P[2];
  mortar_pieces<Real, DIM, N>(G, Mp->m, side, ct, cz, P);
  // lane-dependent piece picked by selects (an indexed access would put the
  // two pieces in private memory)
  const int seg = pc ? P[1].seg : P[0].seg;
  const int jface = pc ? P[1].jface : P[0].jface;
  const CellId other = pc ? P[1].other : P[0].other;
  const CellId C = sd == 0 ? CellId{side, ct, side == 0 ? G.nr[0] - 1 : 0, cz} : other;
  const int cside = sd == 0 ? side : 1 - side;
  Real tg[N][2];  // cos, sin at the piece's points
#pragma unroll
  for (int q = 0; q < N; ++q)
#pragma unroll
    for (int c2 = 0; c2 < 2; ++c2) tg[q][c2] = mtrig[(((size_t)jface * 2 + seg) * N + q) * 2 + c2];
  Real X[EARLY ? NZ : 1][N][N];
  unsigned fixbits = 0;  // constrained entries, applied after the barrier
  if constexpr (EARLY) {
#pragma unroll
    for (int c = 0; c < NZ; ++c)
#pragma unroll
      for (int b2 = 0; b2 < N; ++b2)
#pragma unroll
        for (int a2 = 0; a2 < N; ++a2) {
          int it, ir, iz;
          const long long nd = node_of<Real, DIM>(G, k, C, a2, b2, c, it, ir, iz);
          const bool vfx = vel_fixed<Real, DIM>(G, C.dom, ir, iz), pfx = p_fixed(G, C.dom, it, ir, iz);
          const bool fixed = (mask != 0) & ((m < DIM) ? vfx : pfx);
          X[c][b2][a2] = src[nd * NC + m];
          fixbits |= (fixed ? 1u : 0u) << ((c * N + b2) * N + a2);
        }
  }
  {
    int* dstw = (int*)&M;
#pragma unroll
    for (int j = 0; j < IT; ++j) {
      const int i = (int)threadIdx.x + 64 * j;
      if (i < NW) dstw[i] = w[j];
    }
  }
  __syncthreads();
  {
    if (act) {
      if (sd == 0 && m == 0) {
        // point angles of this piece (one lane per face and piece)
#pragma unroll
        for (int q = 0; q < N; ++q)
#pragma unroll
          for (int c2 = 0; c2 < 2; ++c2) trg[fl][pc][q][c2] = tg[q][c2];
      }
      // r reduction at the interface: F0 = face value, F1 = normal derivative
      Real F0[NZ][N], F1[NZ][N];
#pragma unroll
      for (int c = 0; c < NZ; ++c)
#pragma unroll
        for (int a2 = 0; a2 < N; ++a2) {
          F0[c][a2] = 0;
          F1[c][a2] = 0;
        }
#pragma unroll
      for (int c = 0; c < NZ; ++c)
#pragma unroll
        for (int b2 = 0; b2 < N; ++b2) {
          const Real fv = M.FV[cside][b2], fd = M.FD[cside][b2];
#pragma unroll
          for (int a2 = 0; a2 < N; ++a2) {
            Real x;
            if constexpr (EARLY) {
              x = ((fixbits >> ((c * N + b2) * N + a2)) & 1u) ? Real(0) : X[c][b2][a2];
            } else {
              int it, ir, iz;
              const long long nd = node_of<Real, DIM>(G, k, C, a2, b2, c, it, ir, iz);
              const bool vfx = vel_fixed<Real, DIM>(G, C.dom, ir, iz), pfx = p_fixed(G, C.dom, it, ir, iz);
              const bool fixed = (mask != 0) & ((m < DIM) ? vfx : pfx);
              const Real xv = src[nd * NC + m];
              x = fixed ? Real(0) : xv;
            }
            F0[c][a2] += fv * x;
            F1[c][a2] += fd * x;
          }
        }
      // theta at the piece's points, then z at the Gauss points
#pragma unroll
      for (int qt = 0; qt < N; ++qt) {
        Real G0[NZ], Gt[NZ], Gr[NZ];
#pragma unroll
        for (int c = 0; c < NZ; ++c) {
          Real s0 = 0, st = 0, sr = 0;
#pragma unroll
          for (int a2 = 0; a2 < N; ++a2) {
            const Real mv = M.MV[cside][seg][qt][a2], md = M.MD[cside][seg][qt][a2];
            s0 += mv * F0[c][a2];
            st += md * F0[c][a2];
            sr += mv * F1[c][a2];
          }
          G0[c] = s0;
          Gt[c] = st;
          Gr[c] = sr;
        }
#pragma unroll
        for (int qz = 0; qz < NZ; ++qz) {
          Real v = 0, dt = 0, dr = 0, dz = 0;
#pragma unroll
          for (int c = 0; c < NZ; ++c) {
            const Real vz = (DIM == 3) ? T.V[qz][c] : Real(1);
            const Real dzv = (DIM == 3) ? T.D[qz][c] : Real(0);
            v += vz * G0[c];
            dt += vz * Gt[c];
            dr += vz * Gr[c];
            dz += dzv * G0[c];
          }
          Real* e = &ev[fl][pc][sd][qz * N + qt][m * NE];
          e[0] = v;
          e[1] = dt;
          e[2] = dr;
          if constexpr (DIM == 3) e[3] = dz;
        }
      }
    }
  }
  __syncthreads();
  // ---- phase B: face coefficients of the own side; one lane per (face,
  // point) takes both pieces, so FPB * NQ <= 64 items run in one pass
  const Real nu = G.nu;
  const Real inv_rdth = M.inv_rdth;
  const Real inv_dz = M.inv_dz;
  for (int e = threadIdx.x; e < FPB * NQ; e += blockDim.x) {
    const int fl = e / NQ, q = e % NQ;
    const int fs = mblock * FPB + fl;
    if (fs >= nsides) continue;
    const int side = fs / nfaces, f = fs % nfaces;
    Piece<Real, DIM, N> P[2];
    mortar_pieces<Real, DIM, N>(G, M.m, side, f % G.nth[0], f / G.nth[0], P);
    const int qt = q % N, qz = q / N;
    const Real idr_o = side == 0 ? M.inv_dr[0] : M.inv_dr[1];
    const Real idr_x = side == 0 ? M.inv_dr[1] : M.inv_dr[0];
    const Real tau = side == 0 ? M.tau_pen[0] : M.tau_pen[1];
#pragma unroll
    for (int pc = 0; pc < 2; ++pc) {
      const int seg = pc ? P[1].seg : P[0].seg;
      const Real jxw = M.seg_active[seg] ? M.jxw[seg][qt][(DIM == 3) ? qz : 0] : Real(0);
      const Real cth = trg[fl][pc][qt][0], sth = trg[fl][pc][qt][1];
      Real n[DIM] = {};
      n[0] = side == 0 ? cth : -cth;
      n[1] = side == 0 ? sth : -sth;
      Real Ko[DIM][DIM], Kx[DIM][DIM];
      if constexpr (ISO) {
        using IM = IsoMortarLayout<DIM>;
        const Real* g = iso_mg + ((size_t)(fs * 2 + pc) * NQ + q) * IM::SIZE;
#pragma unroll
        for (int a = 0; a < DIM; ++a)
#pragma unroll
          for (int d2 = 0; d2 < DIM; ++d2) {
            Ko[a][d2] = g[IM::KO + a * DIM + d2];
            Kx[a][d2] = g[IM::KX + a * DIM + d2];
          }
      }
      const Real pbar = Real(0.5) * (ev[fl][pc][0][q][DIM * NE] + ev[fl][pc][1][q][DIM * NE]);
      Real jn = 0;
#pragma unroll
      for (int m = 0; m < DIM; ++m) {
        const Real* eo = &ev[fl][pc][0][q][m * NE];
        const Real* ex = &ev[fl][pc][1][q][m * NE];
        Real gavg[DIM];
        if constexpr (ISO) {
#pragma unroll
          for (int d2 = 0; d2 < DIM; ++d2) {
            Real go = 0, gx = 0;
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
              go += Ko[a][d2] * eo[1 + a];
              gx += Kx[a][d2] * ex[1 + a];
            }
            gavg[d2] = Real(0.5) * (go + gx);
          }
        } else {
          const Real dro = eo[2] * idr_o, dto = eo[1] * inv_rdth;
          const Real drx = ex[2] * idr_x, dtx = ex[1] * inv_rdth;
          gavg[0] = Real(0.5) * ((cth * dro - sth * dto) + (cth * drx - sth * dtx));
          gavg[1] = Real(0.5) * ((sth * dro + cth * dto) + (sth * drx + cth * dtx));
          if constexpr (DIM == 3) gavg[2] = Real(0.5) * (eo[3] + ex[3]) * inv_dz;
        }
        Real gn = 0;
#pragma unroll
        for (int d2 = 0; d2 < DIM; ++d2) gn += gavg[d2] * n[d2];
        const Real j = eo[0] - ex[0];
        jn += j * n[m];
        const Real cv = pbar * n[m] - nu * gn + nu * tau * j;
        Real Gm[DIM];
#pragma unroll
        for (int d2 = 0; d2 < DIM; ++d2) Gm[d2] = Real(-0.5) * nu * j * n[d2];
        Real* cf = &coef[fl][pc][q][m * NE];
        cf[0] = jxw * cv;
        if constexpr (ISO) {
#pragma unroll
          for (int a = 0; a < DIM; ++a) {
            Real t = 0;
#pragma unroll
            for (int d2 = 0; d2 < DIM; ++d2) t += Ko[a][d2] * Gm[d2];
            cf[1 + a] = jxw * t;
          }
        } else {
          cf[1] = jxw * (-sth * Gm[0] + cth * Gm[1]) * inv_rdth;
          cf[2] = jxw * (cth * Gm[0] + sth * Gm[1]) * idr_o;
          if constexpr (DIM == 3) cf[3] = jxw * Gm[2] * inv_dz;
        }
      }
      Real* cf = &coef[fl][pc][q][DIM * NE];
      cf[0] = jxw * Real(-0.5) * jn;
#pragma unroll
      for (int j = 1; j < NE; ++j) cf[j] = 0;
    }
  }
  __syncthreads();
  // ---- phase C: integration against the own cell's test functions; lane =
  // (face, component, z node c): z reverse for its c, theta reverse, then the
  // r expansion to all N rows of the face's cell layer
  for (int e = threadIdx.x; e < FPB * NC * NZ; e += blockDim.x) {
    const int fl = e / (NC * NZ), m = (e / NZ) % NC, c = e % NZ;
    const int fs = mblock * FPB + fl;
    if (fs >= nsides) continue;
    const int side = fs / nfaces, f = fs % nfaces;
    Piece<Real, DIM, N> P[2];
    mortar_pieces<Real, DIM, N>(G, M.m, side, f % G.nth[0], f / G.nth[0], P);
    Real k0[N], k1[N];
#pragma unroll
    for (int a2 = 0; a2 < N; ++a2) {
      k0[a2] = 0;
      k1[a2] = 0;
    }
#pragma unroll
    for (int pc = 0; pc < 2; ++pc) {
      const int seg = pc ? P[1].seg : P[0].seg;
      // z reverse at node c: H0 (value + z-derivative terms), Ht, Hr per qt
      Real H0[N], Ht[N], Hr[N];
#pragma unroll
      for (int qt = 0; qt < N; ++qt) {
        Real h0 = 0, ht = 0, hr = 0;
#pragma unroll
        for (int qz = 0; qz < NZ; ++qz) {
          const Real* cf = &coef[fl][pc][qz * N + qt][m * NE];
          const Real vz = (DIM == 3) ? T.V[qz][c] : Real(1);
          const Real dzv = (DIM == 3) ? T.D[qz][c] : Real(0);
          h0 += vz * cf[0] + ((DIM == 3) ? dzv * cf[3] : Real(0));
          ht += vz * cf[1];
          hr += vz * cf[2];
        }
        H0[qt] = h0;
        Ht[qt] = ht;
        Hr[qt] = hr;
      }
      // theta reverse
#pragma unroll
      for (int a2 = 0; a2 < N; ++a2) {
        Real s0 = 0, s1 = 0;
#pragma unroll
        for (int qt = 0; qt < N; ++qt) {
          const Real mv = M.MV[side][seg][qt][a2], md = M.MD[side][seg][qt][a2];
          s0 += mv * H0[qt] + md * Ht[qt];
          s1 += mv * Hr[qt];
        }
        k0[a2] += s0;
        k1[a2] += s1;
      }
    }
    // r expansion: row b2 takes the face value L_b2 and normal derivative L_b2'
#pragma unroll
    for (int b2 = 0; b2 < N; ++b2) {
      const Real fv = M.FV[side][b2], fd = M.FD[side][b2];
#pragma unroll
      for (int a2 = 0; a2 < N; ++a2)
        Em[(size_t)(m * S::NPT + c * S::PLANE + b2 * N + a2) * nsides + fs] = fv * k0[a2] + fd * k1[a2];
    }
  }
}

template <typename Real, int DIM, int N, bool ISO = false>
__global__ __launch_bounds__(64) void k_mortar(Geom<Real> G, Tab1D<Real, N> T, int k,
                                               const MortarTab<Real, N>* __restrict__ Mp,
                                               const Real* __restrict__ mtrig, const Real* __restrict__ src,
                                               Real* __restrict__ Em, int mask, const Real* __restrict__ iso_mg) {
  __shared__ MortarSmem<Real, DIM, N> sm;
  mortar_block<Real, DIM, N, 36000, ISO>(G, T, k, blockIdx.x, Mp, mtrig, src, Em, mask, sm, iso_mg);
}

// Fused launch: blocks [0, nmb) integrate mortar faces, the rest integrate
// volume cells; the two block kinds share one LDS allocation.
template <typename Real, int DIM, int N, bool ISO = false>
union FusedSmem {
  VolumeSmem<Real, DIM, N, ISO> v;
  MortarSmem<Real, DIM, N> m;
};

template <typename Real, int DIM, int N, bool ISO = false>
__global__ __launch_bounds__(64) void k_jacobian_fused(Geom<Real> G, Tab1D<Real, N> T, int k, int nmb,
                                                                    const Real* __restrict__ lin,
                                                                    const MortarTab<Real, N>* __restrict__ Mp,
                                                                    const Real* __restrict__ mtrig,
                                                                    const Real* __restrict__ src,
                                                                    Real* __restrict__ E, Real* __restrict__ Em,
                                                                    const Real* __restrict__ iso_mg) {
  __shared__ FusedSmem<Real, DIM, N, ISO> sm;
  if ((int)blockIdx.x < nmb)
    mortar_block<Real, DIM, N, 36000, ISO>(G, T, k, blockIdx.x, Mp, mtrig, src, Em, 1, sm.m, iso_mg);
  else volume_block<Real, DIM, N, ISO>(G, T, k, blockIdx.x - nmb, lin, src, E, sm.v);
}

// fused launch with the quad volume layout (3D)
template <typename Real, int N, bool LINC = false>
__global__ __launch_bounds__(64) void k_jacobian_fused_quad(Geom<Real> G, Tab1D<Real, N> T, int k, int nmb,
                                                            const Real* __restrict__ lin,
                                                            const MortarTab<Real, N>* __restrict__ Mp,
                                                            const Real* __restrict__ mtrig,
                                                            const Real* __restrict__ src, Real* __restrict__ E,
                                                            Real* __restrict__ Em, int strip,
                                                            const Real* __restrict__ state, int picard) {
  __shared__ MortarSmem<Real, 3, N> sm;
  // degree 2: volume blocks first, mortar blocks last (FP32 vmult 32.3 ->
  // 28.0 us at 1.1M DoFs); degree 3: mortar blocks first (2 % faster there)
  constexpr bool kVolumeFirst = N == 3;
  const int nvb = (int)gridDim.x - nmb;
  const bool mortar = kVolumeFirst ? (int)blockIdx.x >= nvb : (int)blockIdx.x < nmb;
  if (mortar) mortar_block<Real, 3, N>(G, T, k, kVolumeFirst ? blockIdx.x - nvb : blockIdx.x, Mp, mtrig, src, Em, 1, sm);
  else volume_quad<Real, N, false, LINC>(G, T, k, kVolumeFirst ? blockIdx.x : blockIdx.x - nmb, lin, src, E,
                                         strip != 0, nullptr, state, picard);
}

// Fused launch of the FP64 quad layout with LDS-staged volume blocks: the
// volume blocks keep their point values in the block's LDS and the mortar
// blocks take fewer faces per block, so that both fit the LDS of two
// wavefronts per SIMD (the kernel's registers allow two).
constexpr int kLdsQuadBytes = 4 * 3 * 3 * 64 * 8;  // 3D Q2 FP64 point values
template <int N, bool LINC = false>
__global__ __launch_bounds__(64) void k_jacobian_fused_quad_lds(Geom<double> G, Tab1D<double, N> T, int k, int nmb,
                                                                const double* __restrict__ lin,
                                                                const MortarTab<double, N>* __restrict__ Mp,
                                                                const double* __restrict__ mtrig,
                                                                const double* __restrict__ src,
                                                                double* __restrict__ E, double* __restrict__ Em,
                                                                int strip, const double* __restrict__ state,
                                                                int picard) {
  using MSm = MortarSmem<double, 3, N, kLdsQuadBytes>;
  constexpr int UB = (LINC ? 7 : 4) * N * N * 64 * (int)sizeof(double);
  constexpr int SB = (int)sizeof(MSm) > UB ? (int)sizeof(MSm) : UB;
  __shared__ __align__(16) unsigned char smem[SB];
  // volume blocks first, the mortar blocks last (measured faster than mortar
  // first or alternating)
  const int nvb = (int)gridDim.x - nmb;
  if ((int)blockIdx.x >= nvb)
    mortar_block<double, 3, N, kLdsQuadBytes>(G, T, k, blockIdx.x - nvb, Mp, mtrig, src, Em, 1,
                                              *reinterpret_cast<MSm*>(smem));
  else
    volume_quad<double, N, true, LINC>(G, T, k, blockIdx.x, lin, src, E, strip != 0, reinterpret_cast<double*>(smem),
                                       state, picard);
}

// Mortar part of the diagonal, Alg. Alg-diagonal: the unit vector of own DoF
// i (other side zero) gives, tested with the same basis function,
// nu tau phi^2 - nu phi (grad phi . n) for velocity rows and 0 for pressure rows.
template <typename Real, int DIM, int N>
__global__ __launch_bounds__(64) void k_mortar_diag(Geom<Real> G, Tab1D<Real, N> T, int k,
                                                    const MortarTab<Real, N>* __restrict__ Mp,
                                                    const Real* __restrict__ mtrig, Real* __restrict__ diag) {
  using S = Shape<Real, DIM, N>;
  constexpr int NC = S::NC, NPT = S::NPT, NZ = S::NZ;
  const MortarTab<Real, N>& M = *Mp;
  const int nfaces = G.nth[0] * G.nz;  // equal counts on both sides
  const int side = blockIdx.x / nfaces;
  const int f = blockIdx.x % nfaces;
  const int ct = f % G.nth[0], cz = f / G.nth[0];
  const CellId own{side, ct, side == 0 ? G.nr[0] - 1 : 0, cz};
  Piece<Real, DIM, N> P[2];
  mortar_pieces<Real, DIM, N>(G, M.m, side, ct, cz, P);
  const Real nu = G.nu, tau = M.tau_pen[side];
  for (int node = threadIdx.x; node < NPT; node += blockDim.x) {
    const int a = node % N, b = (node / N) % N, c = node / S::PLANE;
    const Real fv = M.FV[side][b], fd = M.FD[side][b];
    if (fv == Real(0) && fd == Real(0)) continue;
    Real acc[DIM] = {};
    for (int pc = 0; pc < 2; ++pc) {
      const int seg = pc ? P[1].seg : P[0].seg;
      if (!M.seg_active[seg]) continue;
      for (int qz = 0; qz < NZ; ++qz)
        for (int qt = 0; qt < N; ++qt) {
          const Real vz = (DIM == 3) ? T.V[qz][c] : Real(1);
          const Real mv = M.MV[side][seg][qt][a];
          const Real phi = mv * fv * vz;
          const Real dr = mv * fd * vz / G.dr[side];
          // grad phi . n with n = +-e_r is +-(d phi / dr)
          const Real gn = side == 0 ? dr : -dr;
          const Real jxw = M.jxw[seg][qt][(DIM == 3) ? qz : 0];
          const Real v = jxw * (nu * tau * phi * phi - nu * phi * gn);
#pragma unroll
          for (int m = 0; m < DIM; ++m) acc[m] += v;
        }
    }
    int it, ir, iz;
    const long long nd = node_of<Real, DIM>(G, k, own, a, b, c, it, ir, iz);
#pragma unroll
    for (int m = 0; m < DIM; ++m) atomic_add(diag + nd * NC + m, acc[m]);
  }
}

// ---------------------------------------------------------------------------
// Mortar face terms with unequal interface counts (the restriction of
// Sec. 3.1 lifted, as Sec. 5 proposes): a face of one side meets every face
// of the other side that overlaps it, and each intersection is one segment
// with the Gauss rule of Sec. 3.2 mapped into it (JxW = w R dtheta_seg dz).
// One 64-lane block per interface face side (rotor faces first); for every
// segment of its face:
//   - the other cell's nodal values join the own cell's in LDS;
//   - lane per (point, component, side): value and reference derivatives at
//     the point, by direct sums over the cell's nodes (the theta basis at the
//     segment's points evaluated in FP64 from the Gauss-Lobatto nodes);
//   - lane per point: the own side's face coefficients (jump = own - other,
//     n = own outward normal) times JxW;
//   - lane per (own local node, component): the test integrals, summed over
//     the segments in registers and stored once, Em[comp][local node][face side].
// Segments shorter than 1e-12 of the smaller cell angle are dropped (the
// alignment rule of the equal-count tables).
// ---------------------------------------------------------------------------
constexpr int kMaxPieces = 6;  // segments per face: ceil(4) + 2 for ring counts at most 4:1 apart

template <int N>
__device__ inline void lagrange_gll(const MortarGen& MG, double t, double (&L)[N], double (&dL)[N]) {
#pragma unroll
  for (int j = 0; j < N; ++j) {
    double p = 1.0, dp = 0.0;
#pragma unroll
    for (int q = 0; q < N; ++q) {
      if (q == j) continue;
      const double inv = MG.ginv[j][q];
      const double f = (t - MG.gll[q]) * inv;
      dp = dp * f + p * inv;
      p = p * f;
    }
    L[j] = p;
    dL[j] = dp;
  }
}

// the face of side `side` with ring index ct: cell angle, start angle and
// the position of its start in the other side's ring, reduced to [0, 2 pi)
struct GenFace {
  double dth_s, dth_o, start, delta, tol;
  int nto, f0;
};

template <typename Real>
__device__ inline GenFace gen_face(const Geom<Real>& G, const MortarGen& MG, int side, int ct) {
  constexpr double kTwoPi = 6.283185307179586476925286766559;
  GenFace F;
  const int nts = pick(side, G.nth);
  F.nto = pick(1 - side, G.nth);
  F.dth_s = kTwoPi / nts;
  F.dth_o = kTwoPi / F.nto;
  const double th0_s = side == 0 ? MG.theta_rot : 0.0, th0_o = side == 0 ? 0.0 : MG.theta_rot;
  F.start = th0_s + ct * F.dth_s;
  double delta = fmod(F.start - th0_o, kTwoPi);
  if (delta < 0) delta += kTwoPi;
  F.delta = delta;
  F.tol = 1e-12 * fmin(F.dth_s, F.dth_o);
  F.f0 = (int)floor(delta / F.dth_o);
  return F;
}

// inverse of the reference-to-physical Jacobian J[m][p] = d x_m / d xi_p:
// K[p][m] = d xi_p / d x_m
template <int DIM>
__device__ inline void invert_jacobian(const double (&J)[DIM][DIM], double (&K)[DIM][DIM]) {
  if constexpr (DIM == 2) {
    const double id = 1.0 / (J[0][0] * J[1][1] - J[0][1] * J[1][0]);
    K[0][0] = J[1][1] * id;
    K[0][1] = -J[0][1] * id;
    K[1][0] = -J[1][0] * id;
    K[1][1] = J[0][0] * id;
  } else {
    const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    const double id = 1.0 / (J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02);
    K[0][0] = c00 * id;
    K[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * id;
    K[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * id;
    K[1][0] = c01 * id;
    K[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * id;
    K[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * id;
    K[2][0] = c02 * id;
    K[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * id;
    K[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * id;
  }
}

// position of node nd in the current configuration (rotor nodes rotated by
// the rotor angle, Sec. 3.1)
__device__ inline void node_position(const double* __restrict__ xnode, long long nd, bool rotor, double c, double s,
                                     double (&x)[3]) {
  const double x0 = xnode[nd * 3], y0 = xnode[nd * 3 + 1];
  x[0] = rotor ? c * x0 - s * y0 : x0;
  x[1] = rotor ? s * x0 + c * y0 : y0;
  x[2] = xnode[nd * 3 + 2];
}

// ISO: iso-parametric cells; the gradients at the mortar points go through
// each side's inverse Jacobian there, read with the points' angles from the
// table of the current rotor angle (MG.iso_geo; the mortar points, JxW and
// normals stay those of the exact circle)
template <typename Real, int DIM, int N, bool ISO = false>
__global__ __launch_bounds__(64) void k_mortar_general(Geom<Real> G, Tab1D<Real, N> T, int k, MortarGen MG,
                                                       const Real* __restrict__ src, Real* __restrict__ Em,
                                                       int mask) {
  using S = Shape<Real, DIM, N>;
  using IM = IsoMortarLayout<DIM>;
  constexpr int NC = S::NC, NPT = S::NPT, NZ = S::NZ, NQ = N * NZ, NE = DIM + 1;
  constexpr int NI = (NPT * NC + 63) / 64;
  __shared__ Real U[2][NC][NPT];    // nodal values: own cell (0), other cell (1)
  __shared__ Real ev[2][NQ][NC][NE];// value, d/dxi_theta, d/dxi_r, d/dxi_z at the points
  __shared__ Real cf[NQ][NC][NE];   // own-side test coefficients times JxW
  __shared__ Real Lt[2][N][N], dLt[2][N][N];  // theta basis of both sides at the segment's points [side][qt][a]
  const int tid = threadIdx.x;
  const int nf0 = G.nth[0] * G.nz;
  const int nsides = nf0 + G.nth[1] * G.nz;
  const int fs = blockIdx.x;
  const int side = fs >= nf0;
  const int f = side ? fs - nf0 : fs;
  const int nts = pick(side, G.nth);
  const int ct = f % nts, cz = f / nts;
  const int cr_own = side == 0 ? G.nr[0] - 1 : 0, cr_oth = side == 0 ? 0 : G.nr[0] - 1;
  const CellId own{side, ct, cr_own, cz};
  const GenFace F = gen_face(G, MG, side, ct);
  auto load_cell = [&](const CellId& C, int slot) {
    for (int e = tid; e < NPT * NC; e += 64) {
      const int node = e / NC, m = e % NC;
      const int a = node % N, b = (node / N) % N, c = node / S::PLANE;
      int it, ir, iz;
      const long long nd = node_of<Real, DIM>(G, k, C, a, b, c, it, ir, iz);
      const bool fixed = (mask != 0) & ((m < DIM) ? vel_fixed<Real, DIM>(G, C.dom, ir, iz) : p_fixed(G, C.dom, it, ir, iz));
      U[slot][m][node] = fixed ? Real(0) : src[nd * NC + m];
    }
  };
  load_cell(own, 0);
  Real acc[NI];
#pragma unroll
  for (int i = 0; i < NI; ++i) acc[i] = 0;
  const Real nu = G.nu;
  const double R = MG.R;
  const double idr_s = MG.inv_dr[side], idr_o = MG.inv_dr[1 - side];
  const double irdth_s = 1.0 / (R * F.dth_s), irdth_o = 1.0 / (R * F.dth_o);
  const double tau = MG.tau_pen[side];
  for (int p = 0; p < kMaxPieces; ++p) {
    const int fo = F.f0 + p;
    const double a_f = fo * F.dth_o - F.delta;  // other face start, in the own face's local angle
    if (a_f >= F.dth_s - F.tol) break;
    if (ISO && p >= MG.npiece) break;  // the table's slots bound the segments of a face
    const double lo = fmax(0.0, a_f), hi = fmin(F.dth_s, a_f + F.dth_o);
    if (hi - lo <= F.tol) continue;
    const int ofc = ((fo % F.nto) + F.nto) % F.nto;
    const CellId oth{1 - side, ofc, cr_oth, cz};
    __syncthreads();  // the previous segment is done with U[1], ev, cf, Lt
    load_cell(oth, 1);
    // theta basis of both sides at the segment's points
    for (int i = tid; i < 2 * N; i += 64) {
      const int sd = i / N, qt = i % N;
      const double sl = lo + (double)T.x[qt] * (hi - lo);
      double L[N], dL[N];
      lagrange_gll<N>(MG, sd == 0 ? sl / F.dth_s : (sl - a_f) / F.dth_o, L, dL);
#pragma unroll
      for (int a = 0; a < N; ++a) {
        Lt[sd][qt][a] = (Real)L[a];
        dLt[sd][qt][a] = (Real)dL[a];
      }
    }
    __syncthreads();
    // evaluation at the segment's points
    for (int e = tid; e < 2 * NQ * NC; e += 64) {
      const int sd = e / (NQ * NC), q = (e / NC) % NQ, m = e % NC;
      const int qt = q % N, qz = q / N;
      const int cs = sd == 0 ? side : 1 - side;
      Real v = 0, dt = 0, dr = 0, dz = 0;
#pragma unroll
      for (int c = 0; c < NZ; ++c) {
        const Real lz = (DIM == 3) ? T.V[qz][c] : Real(1);
        const Real dlz = (DIM == 3) ? T.D[qz][c] : Real(0);
#pragma unroll
        for (int b = 0; b < N; ++b) {
          const Real fv = (Real)MG.FV[cs][b], fd = (Real)MG.FD[cs][b];
          Real s0 = 0, s1 = 0;
#pragma unroll
          for (int a = 0; a < N; ++a) {
            const Real u = U[sd][m][(c * N + b) * N + a];
            s0 += Lt[sd][qt][a] * u;
            s1 += dLt[sd][qt][a] * u;
          }
          v += lz * fv * s0;
          dt += lz * fv * s1;
          dr += lz * fd * s0;
          dz += dlz * fv * s0;
        }
      }
      Real* o = ev[sd][q][m];
      o[0] = v;
      o[1] = dt;
      o[2] = dr;
      if constexpr (DIM == 3) o[3] = dz;
    }
    __syncthreads();
    // the own side's face coefficients at every point
    for (int q = tid; q < NQ; q += 64) {
      const int qt = q % N, qz = q / N;
      const double sl = lo + (double)T.x[qt] * (hi - lo);
      double jxw = (double)T.w[qt] * R * (hi - lo);
      if constexpr (DIM == 3) jxw *= (double)T.w[qz] / MG.inv_dz;
      Real c, sn, Ko[DIM][DIM], Kx[DIM][DIM];
      if constexpr (ISO) {
        const Real* g = (const Real*)MG.iso_geo + ((size_t)(fs * MG.npiece + p) * NQ + q) * IM::SIZE;
#pragma unroll
        for (int a = 0; a < DIM; ++a)
#pragma unroll
          for (int m = 0; m < DIM; ++m) {
            Ko[a][m] = g[IM::KO + a * DIM + m];
            Kx[a][m] = g[IM::KX + a * DIM + m];
          }
        c = g[IM::C];
        sn = g[IM::S];
      } else {
        double sth, cth;
        sincos(F.start + sl, &sth, &cth);
        c = (Real)cth;
        sn = (Real)sth;
      }
      const Real J = (Real)jxw;
      Real n[DIM] = {};
      n[0] = side == 0 ? c : -c;
      n[1] = side == 0 ? sn : -sn;
      const Real pbar = Real(0.5) * (ev[0][q][DIM][0] + ev[1][q][DIM][0]);
      Real jn = 0;
#pragma unroll
      for (int m = 0; m < DIM; ++m) {
        const Real* eo = ev[0][q][m];
        const Real* ex = ev[1][q][m];
        Real gavg[DIM];
        if constexpr (ISO) {
#pragma unroll
          for (int d2 = 0; d2 < DIM; ++d2) {
            Real go = 0, gx = 0;
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
              go += Ko[a][d2] * eo[1 + a];
              gx += Kx[a][d2] * ex[1 + a];
            }
            gavg[d2] = Real(0.5) * (go + gx);
          }
        } else {
          const Real dro = eo[2] * (Real)idr_s, dto = eo[1] * (Real)irdth_s;
          const Real drx = ex[2] * (Real)idr_o, dtx = ex[1] * (Real)irdth_o;
          gavg[0] = Real(0.5) * ((c * dro - sn * dto) + (c * drx - sn * dtx));
          gavg[1] = Real(0.5) * ((sn * dro + c * dto) + (sn * drx + c * dtx));
          if constexpr (DIM == 3) gavg[2] = Real(0.5) * (eo[3] + ex[3]) * (Real)MG.inv_dz;
        }
        Real gn = 0;
#pragma unroll
        for (int d2 = 0; d2 < DIM; ++d2) gn += gavg[d2] * n[d2];
        const Real j = eo[0] - ex[0];
        jn += j * n[m];
        const Real cv = pbar * n[m] - nu * gn + nu * (Real)tau * j;
        Real Gm[DIM];
#pragma unroll
        for (int d2 = 0; d2 < DIM; ++d2) Gm[d2] = Real(-0.5) * nu * j * n[d2];
        Real* o = cf[q][m];
        o[0] = J * cv;
        if constexpr (ISO) {
#pragma unroll
          for (int a = 0; a < DIM; ++a) {
            Real t = 0;
#pragma unroll
            for (int d2 = 0; d2 < DIM; ++d2) t += Ko[a][d2] * Gm[d2];
            o[1 + a] = J * t;
          }
        } else {
          o[1] = J * (-sn * Gm[0] + c * Gm[1]) * (Real)irdth_s;
          o[2] = J * (c * Gm[0] + sn * Gm[1]) * (Real)idr_s;
          if constexpr (DIM == 3) o[3] = J * Gm[2] * (Real)MG.inv_dz;
        }
      }
      Real* o = cf[q][DIM];
      o[0] = J * Real(-0.5) * jn;
#pragma unroll
      for (int j = 1; j < NE; ++j) o[j] = 0;
    }
    __syncthreads();
    // test integrals of the own cell's basis functions
#pragma unroll
    for (int ii = 0; ii < NI; ++ii) {
      const int e = tid + 64 * ii;
      const int node = (e < NPT * NC ? e : 0) / NC, m = e % NC;
      const int a = node % N, b = (node / N) % N, c = node / S::PLANE;
      const Real fv = (Real)MG.FV[side][b], fd = (Real)MG.FD[side][b];
      Real sum = 0;
      for (int q = 0; q < NQ; ++q) {
        const int qt = q % N, qz = q / N;
        const Real lz = (DIM == 3) ? T.V[qz][c] : Real(1);
        const Real dlz = (DIM == 3) ? T.D[qz][c] : Real(0);
        const Real lt = Lt[0][qt][a], dlt = dLt[0][qt][a];
        const Real* o = cf[q][m];
        sum += o[0] * lt * fv * lz + o[1] * dlt * fv * lz + o[2] * lt * fd * lz;
        if constexpr (DIM == 3) sum += o[3] * lt * fv * dlz;
      }
      acc[ii] += sum;
    }
  }
#pragma unroll
  for (int ii = 0; ii < NI; ++ii) {
    const int e = tid + 64 * ii;
    const int node = e / NC, m = e % NC;
    if (e < NPT * NC) Em[(size_t)(m * NPT + node) * nsides + fs] = acc[ii];
  }
}

// Mortar point geometry of an iso-parametric interface at the current rotor
// angle (IsoMortarLayout): one block per face side; per segment, point and
// side the Jacobian of the cell's interpolated map from its node positions
// (rotor nodes rotated), inverted.  Segment order: with equal ring counts
// that of mortar_block (two pieces per face, segments of phi = theta mod
// dtheta, f = phi / dtheta, offset mstep), else that of k_mortar_general.
template <int DIM, int N>
__global__ __launch_bounds__(64) void k_iso_mortar_geo(Geom<double> G, Tab1D<double, N> T, int k, MortarGen MG,
                                                       int polar_order, int mstep, double f_phi,
                                                       double* __restrict__ g64, float* __restrict__ g32) {
  using S = Shape<double, DIM, N>;
  using IM = IsoMortarLayout<DIM>;
  constexpr int NPT = S::NPT, NZ = S::NZ, NQ = N * NZ;
  __shared__ double X[2][3][NPT];
  __shared__ double Lt[2][N][N], dLt[2][N][N];
  __shared__ double ang[N];
  const int tid = threadIdx.x;
  const int nf0 = G.nth[0] * G.nz;
  const int fs = blockIdx.x;
  const int side = fs >= nf0;
  const int f = side ? fs - nf0 : fs;
  const int nts = pick(side, G.nth);
  const int ct = f % nts, cz = f / nts;
  const int cr_own = side == 0 ? G.nr[0] - 1 : 0, cr_oth = side == 0 ? 0 : G.nr[0] - 1;
  const GenFace F = gen_face(G, MG, side, ct);
  double crot, srot;
  sincos(MG.theta_rot, &srot, &crot);
  auto load_x = [&](const CellId& C, int slot) {
    for (int node = tid; node < NPT; node += 64) {
      const int a = node % N, b = (node / N) % N, c = node / S::PLANE;
      int it, ir, iz;
      const long long nd = node_of<double, DIM>(G, k, C, a, b, c, it, ir, iz);
      double x[3];
      node_position(MG.xnode, nd, C.dom == 0, crot, srot, x);
#pragma unroll
      for (int m = 0; m < 3; ++m) X[slot][m][node] = x[m];
    }
  };
  load_x(CellId{side, ct, cr_own, cz}, 0);
  Piece<double, DIM, N> P[2];
  if (polar_order) mortar_pieces<double, DIM, N>(G, mstep, side, ct, cz, P);
  const double dth = F.dth_s;
  for (int p = 0; p < kMaxPieces && p < MG.npiece; ++p) {
    CellId oth;
    double lo = 0, hi = 0, a_f = 0;
    int seg = 0, jface = 0;
    if (polar_order) {
      if (p >= 2) break;
      seg = P[p].seg;
      jface = P[p].jface;
      oth = P[p].other;
    } else {
      const int fo = F.f0 + p;
      a_f = fo * F.dth_o - F.delta;
      if (a_f >= F.dth_s - F.tol) break;
      lo = fmax(0.0, a_f);
      hi = fmin(F.dth_s, a_f + F.dth_o);
      if (hi - lo <= F.tol) continue;
      oth = CellId{1 - side, ((fo % F.nto) + F.nto) % F.nto, cr_oth, cz};
    }
    __syncthreads();
    load_x(oth, 1);
    for (int i = tid; i < 2 * N; i += 64) {
      const int sd = i / N, qt = i % N;
      const double t = T.x[qt];
      double xi;
      if (polar_order) {
        // reference coordinate of the stator (s) and rotor (r) cell at the
        // point, as in the mortar tables of the rotation
        const double xs = seg == 0 ? t * f_phi : f_phi + t * (1.0 - f_phi);
        const double xr = seg == 0 ? 1.0 - f_phi + t * f_phi : t * (1.0 - f_phi);
        const int cs = sd == 0 ? side : 1 - side;
        xi = cs == 1 ? xs : xr;
        if (sd == 0) ang[qt] = (jface + xs) * dth;
      } else {
        const double sl = lo + t * (hi - lo);
        xi = sd == 0 ? sl / F.dth_s : (sl - a_f) / F.dth_o;
        if (sd == 0) ang[qt] = F.start + sl;
      }
      double L[N], dL[N];
      lagrange_gll<N>(MG, xi, L, dL);
#pragma unroll
      for (int a = 0; a < N; ++a) {
        Lt[sd][qt][a] = L[a];
        dLt[sd][qt][a] = dL[a];
      }
    }
    __syncthreads();
    for (int e = tid; e < 2 * NQ; e += 64) {
      const int sd = e / NQ, q = e % NQ;
      const int qt = q % N, qz = q / N;
      const int cs = sd == 0 ? side : 1 - side;
      double J[DIM][DIM];
#pragma unroll
      for (int m = 0; m < DIM; ++m) {
        double dt = 0, dr = 0, dz = 0;
        for (int c = 0; c < NZ; ++c) {
          const double lz = (DIM == 3) ? T.V[qz][c] : 1.0;
          const double dlz = (DIM == 3) ? T.D[qz][c] : 0.0;
          for (int b = 0; b < N; ++b) {
            double s0 = 0, s1 = 0;
#pragma unroll
            for (int a = 0; a < N; ++a) {
              const double x = X[sd][m][(c * N + b) * N + a];
              s0 += Lt[sd][qt][a] * x;
              s1 += dLt[sd][qt][a] * x;
            }
            dt += lz * MG.FV[cs][b] * s1;
            dr += lz * MG.FD[cs][b] * s0;
            dz += dlz * MG.FV[cs][b] * s0;
          }
        }
        J[m][0] = dt;
        J[m][1] = dr;
        if constexpr (DIM == 3) J[m][2] = dz;
      }
      double K[DIM][DIM];
      invert_jacobian<DIM>(J, K);
      const size_t o = ((size_t)(fs * MG.npiece + p) * NQ + q) * IM::SIZE;
      const int off = sd == 0 ? IM::KO : IM::KX;
#pragma unroll
      for (int a = 0; a < DIM; ++a)
#pragma unroll
        for (int m = 0; m < DIM; ++m) {
          g64[o + off + a * DIM + m] = K[a][m];
          g32[o + off + a * DIM + m] = (float)K[a][m];
        }
      if (sd == 0) {
        double sth, cth;
        sincos(ang[qt], &sth, &cth);
        g64[o + IM::C] = cth;
        g64[o + IM::S] = sth;
        g32[o + IM::C] = (float)cth;
        g32[o + IM::S] = (float)sth;
      }
    }
  }
}

// Mortar part of the diagonal with unequal interface counts (Alg.
// Alg-diagonal): the unit vector of own DoF i (other side zero) tested with
// the same basis function gives nu tau phi^2 - nu phi (grad phi . n) for
// velocity rows, 0 for pressure rows, summed over the face's segments.
template <typename Real, int DIM, int N>
__global__ __launch_bounds__(64) void k_mortar_diag_general(Geom<Real> G, Tab1D<Real, N> T, int k, MortarGen MG,
                                                            Real* __restrict__ diag) {
  using S = Shape<Real, DIM, N>;
  constexpr int NC = S::NC, NPT = S::NPT, NZ = S::NZ;
  const int nf0 = G.nth[0] * G.nz;
  const int fs = blockIdx.x;
  const int side = fs >= nf0;
  const int f = side ? fs - nf0 : fs;
  const int nts = pick(side, G.nth);
  const int ct = f % nts, cz = f / nts;
  const CellId own{side, ct, side == 0 ? G.nr[0] - 1 : 0, cz};
  const GenFace F = gen_face(G, MG, side, ct);
  const double nu = (double)G.nu, tau = MG.tau_pen[side], idr = MG.inv_dr[side];
  for (int node = threadIdx.x; node < NPT; node += blockDim.x) {
    const int a = node % N, b = (node / N) % N, c = node / S::PLANE;
    const double fv = MG.FV[side][b], fd = MG.FD[side][b];
    double acc = 0;
    for (int p = 0; p < kMaxPieces; ++p) {
      const double a_f = (F.f0 + p) * F.dth_o - F.delta;
      if (a_f >= F.dth_s - F.tol) break;
      const double lo = fmax(0.0, a_f), hi = fmin(F.dth_s, a_f + F.dth_o);
      if (hi - lo <= F.tol) continue;
      for (int qz = 0; qz < NZ; ++qz)
        for (int qt = 0; qt < N; ++qt) {
          double L[N], dL[N];
          lagrange_gll<N>(MG, (lo + (double)T.x[qt] * (hi - lo)) / F.dth_s, L, dL);
          const double vz = (DIM == 3) ? (double)T.V[qz][c] : 1.0;
          double jxw = (double)T.w[qt] * MG.R * (hi - lo);
          if (DIM == 3) jxw *= (double)T.w[qz] / MG.inv_dz;
          const double phi = L[a] * fv * vz;
          const double dr = L[a] * fd * vz * idr;
          const double gn = side == 0 ? dr : -dr;  // grad phi . n, n = +-e_r
          acc += jxw * (nu * tau * phi * phi - nu * phi * gn);
        }
    }
    int it, ir, iz;
    const long long nd = node_of<Real, DIM>(G, k, own, a, b, c, it, ir, iz);
#pragma unroll
    for (int m = 0; m < DIM; ++m) atomic_add(diag + nd * NC + m, (Real)acc);
  }
}

// The same on iso-parametric cells: grad phi . n through the inverse
// Jacobian of the own cell's interpolated map at each mortar point, which is
// formed once per point in LDS from the cell's node positions.
template <typename Real, int DIM, int N>
__global__ __launch_bounds__(64) void k_mortar_diag_iso(Geom<Real> G, Tab1D<Real, N> T, int k, MortarGen MG,
                                                        Real* __restrict__ diag) {
  using S = Shape<Real, DIM, N>;
  constexpr int NC = S::NC, NPT = S::NPT, NZ = S::NZ, NQ = N * NZ;
  constexpr int NI = (NPT + 63) / 64;
  __shared__ double X[3][NPT];
  __shared__ double Kq[NQ][DIM][DIM];
  __shared__ double Lq[NQ][N], dLq[NQ][N];  // own theta basis at the points
  const int tid = threadIdx.x;
  const int nf0 = G.nth[0] * G.nz;
  const int fs = blockIdx.x;
  const int side = fs >= nf0;
  const int f = side ? fs - nf0 : fs;
  const int nts = pick(side, G.nth);
  const int ct = f % nts, cz = f / nts;
  const CellId own{side, ct, side == 0 ? G.nr[0] - 1 : 0, cz};
  const GenFace F = gen_face(G, MG, side, ct);
  double crot, srot;
  sincos(MG.theta_rot, &srot, &crot);
  for (int node = tid; node < NPT; node += 64) {
    const int a = node % N, b = (node / N) % N, c = node / S::PLANE;
    int it, ir, iz;
    const long long nd = node_of<Real, DIM>(G, k, own, a, b, c, it, ir, iz);
    double x[3];
    node_position(MG.xnode, nd, side == 0, crot, srot, x);
#pragma unroll
    for (int m = 0; m < 3; ++m) X[m][node] = x[m];
  }
  const double nu = (double)G.nu, tau = MG.tau_pen[side];
  const double sgn = side == 0 ? 1.0 : -1.0;  // n = +-e_r
  double acc[NI];
#pragma unroll
  for (int i = 0; i < NI; ++i) acc[i] = 0;
  for (int p = 0; p < kMaxPieces; ++p) {
    const double a_f = (F.f0 + p) * F.dth_o - F.delta;
    if (a_f >= F.dth_s - F.tol) break;
    const double lo = fmax(0.0, a_f), hi = fmin(F.dth_s, a_f + F.dth_o);
    if (hi - lo <= F.tol) continue;
    __syncthreads();  // X loaded; the previous piece is done with Kq, Lq
    for (int q = tid; q < NQ; q += 64) {
      const int qt = q % N, qz = q / N;
      double L[N], dL[N];
      lagrange_gll<N>(MG, (lo + (double)T.x[qt] * (hi - lo)) / F.dth_s, L, dL);
      double J[DIM][DIM];
#pragma unroll
      for (int m = 0; m < DIM; ++m) {
        double dt = 0, dr = 0, dz = 0;
        for (int c = 0; c < NZ; ++c) {
          const double lz = (DIM == 3) ? (double)T.V[qz][c] : 1.0;
          const double dlz = (DIM == 3) ? (double)T.D[qz][c] : 0.0;
          for (int b = 0; b < N; ++b) {
            double s0 = 0, s1 = 0;
#pragma unroll
            for (int a = 0; a < N; ++a) {
              const double x = X[m][(c * N + b) * N + a];
              s0 += L[a] * x;
              s1 += dL[a] * x;
            }
            dt += lz * MG.FV[side][b] * s1;
            dr += lz * MG.FD[side][b] * s0;
            dz += dlz * MG.FV[side][b] * s0;
          }
        }
        J[m][0] = dt;
        J[m][1] = dr;
        if constexpr (DIM == 3) J[m][2] = dz;
      }
      double K[DIM][DIM];
      invert_jacobian<DIM>(J, K);
#pragma unroll
      for (int a = 0; a < DIM; ++a)
#pragma unroll
        for (int m = 0; m < DIM; ++m) Kq[q][a][m] = K[a][m];
#pragma unroll
      for (int a = 0; a < N; ++a) {
        Lq[q][a] = L[a];
        dLq[q][a] = dL[a];
      }
    }
    __syncthreads();
#pragma unroll
    for (int ii = 0; ii < NI; ++ii) {
      const int node = tid + 64 * ii;
      if (node >= NPT) continue;
      const int a = node % N, b = (node / N) % N, c = node / S::PLANE;
      const double fv = MG.FV[side][b], fd = MG.FD[side][b];
      for (int q = 0; q < NQ; ++q) {
        const int qt = q % N, qz = q / N;
        const double vz = (DIM == 3) ? (double)T.V[qz][c] : 1.0;
        const double dvz = (DIM == 3) ? (double)T.D[qz][c] : 0.0;
        double jxw = (double)T.w[qt] * MG.R * (hi - lo);
        if (DIM == 3) jxw *= (double)T.w[qz] / MG.inv_dz;
        const double phi = Lq[q][a] * fv * vz;
        double dref[3] = {dLq[q][a] * fv * vz, Lq[q][a] * fd * vz, Lq[q][a] * fv * dvz};
        // grad phi . n with n = sgn (cos theta, sin theta) at the point
        double sth, cth;
        sincos(F.start + lo + (double)T.x[qt] * (hi - lo), &sth, &cth);
        double gn = 0;
#pragma unroll
        for (int a2 = 0; a2 < DIM; ++a2) gn += (Kq[q][a2][0] * cth + Kq[q][a2][1] * sth) * dref[a2];
        gn *= sgn;
        acc[ii] += jxw * (nu * tau * phi * phi - nu * phi * gn);
      }
    }
  }
#pragma unroll
  for (int ii = 0; ii < NI; ++ii) {
    const int node = tid + 64 * ii;
    if (node >= NPT) continue;
    const int a = node % N, b = (node / N) % N, c = node / S::PLANE;
    int it, ir, iz;
    const long long nd = node_of<Real, DIM>(G, k, own, a, b, c, it, ir, iz);
#pragma unroll
    for (int m = 0; m < DIM; ++m) atomic_add(diag + nd * NC + m, (Real)acc[ii]);
  }
}

// ---------------------------------------------------------------------------
// small vector kernels
// ---------------------------------------------------------------------------
template <typename Real>
__global__ void k_fill(Real* x, Real v, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long j = i; j < n; j += stride) x[j] = v;
}

// mode 0: dst[c] = src[c]; mode 1: dst[c] = 0; mode 2: dst[c] = value
template <typename Real>
__global__ void k_constraints(const int64_t* __restrict__ cons, long long n, const Real* __restrict__ src,
                              Real* __restrict__ dst, Real value, int mode) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t c = cons[i];
  dst[c] = mode == 0 ? src[c] : (mode == 1 ? Real(0) : value);
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
template <typename Real, int N>
static Tab1D<Real, N> make_tab(const mns_handle* h) {
  Tab1D<Real, N> T;
  std::vector<double> L(N), dL(N), d2L(N);
  for (int q = 0; q < N; ++q) {
    lagrange_1d(h->gll, h->gx[q], L.data(), dL.data(), d2L.data());
    for (int a = 0; a < N; ++a) {
      T.V[q][a] = (Real)L[a];
      T.D[q][a] = (Real)dL[a];
      T.DD[q][a] = (Real)d2L[a];
    }
    lagrange_1d(h->gx, h->gx[q], L.data(), dL.data(), d2L.data());
    for (int j = 0; j < N; ++j) {
      T.CD[q][j] = (Real)dL[j];
      T.CDD[q][j] = (Real)d2L[j];
    }
    T.x[q] = (Real)h->gx[q];
    T.w[q] = (Real)h->gw[q];
  }
  return T;
}

template <typename Real>
static Geom<Real> make_geom(const mns_handle* h) {
  Geom<Real> G;
  const mns_mesh_desc& d = h->desc;
  G.ncells = h->ncells;
  G.cell_off1 = h->cell_off1;
  G.node_off1 = h->node_off1;
  G.ndofs = h->ndofs;
  G.nth[0] = h->nth[0];
  G.nth[1] = h->nth[1];
  G.ntd[0] = h->ntd[0];
  G.ntd[1] = h->ntd[1];
  G.nz = h->nz;
  G.nzn = h->nzn;
  G.nr[0] = d.n_r_rotor;
  G.nr[1] = d.n_r_stator;
  G.nrn[0] = h->nrn[0];
  G.nrn[1] = h->nrn[1];
  G.r0[0] = (Real)d.r_in;
  G.r0[1] = (Real)d.r_interface;
  G.dr[0] = (Real)((d.r_interface - d.r_in) / d.n_r_rotor);
  G.dr[1] = (Real)((d.r_out - d.r_interface) / d.n_r_stator);
  G.dthd[0] = (Real)h->dthd[0];
  G.dthd[1] = (Real)h->dthd[1];
  G.dz = (Real)h->dz;
  G.nu = (Real)d.nu;
  G.omega = (Real)h->omega;
  G.ct = d.steady ? Real(0) : (Real)(1.5 / d.dt);
  G.ctau2 = d.steady ? Real(0) : (Real)(1.0 / (d.dt * d.dt));
  G.h[0] = G.h[1] = 0;
  G.hstride = h->hstride;
  if constexpr (sizeof(Real) == 8) {
    G.hcell = (const Real*)h->d_hcell64;
    G.trig = (const Real*)h->d_trig64;
    G.geo = h->iso ? (const Real*)h->d_geo64 : nullptr;
  } else {
    G.hcell = (const Real*)h->d_hcell32;
    G.trig = (const Real*)h->d_trig32;
    G.geo = h->iso ? (const Real*)h->d_geo32 : nullptr;
  }
  G.geox = h->iso ? h->d_geox : nullptr;
  G.hiso = h->iso ? h->d_hiso : nullptr;
  return G;
}

// interface data of the general mortar kernels (unequal ring counts)
static MortarGen make_mortar_gen(const mns_handle* h) {
  MortarGen M{};
  const mns_mesh_desc& d = h->desc;
  M.theta_rot = h->theta;
  M.xnode = h->iso ? h->d_xnode : nullptr;
  M.R = d.r_interface;
  M.tau_pen[0] = h->tau_pen[0];
  M.tau_pen[1] = h->tau_pen[1];
  M.inv_dr[0] = 1.0 / ((d.r_interface - d.r_in) / d.n_r_rotor);
  M.inv_dr[1] = 1.0 / ((d.r_out - d.r_interface) / d.n_r_stator);
  M.inv_dz = d.dim == 3 ? 1.0 / h->dz : 0.0;
  std::vector<double> L(h->n), dL(h->n), d2L(h->n);
  for (int i = 0; i < h->n; ++i) M.gll[i] = h->gll[i];
  for (int j = 0; j < h->n; ++j)
    for (int q = 0; q < h->n; ++q) M.ginv[j][q] = j == q ? 0.0 : 1.0 / (h->gll[j] - h->gll[q]);
  M.npiece = h->mgeo_pieces;
  for (int side = 0; side < 2; ++side) {
    lagrange_1d(h->gll, side == 0 ? 1.0 : 0.0, L.data(), dL.data(), d2L.data());
    for (int b = 0; b < h->n; ++b) {
      M.FV[side][b] = L[b];
      M.FD[side][b] = dL[b];
    }
  }
  return M;
}

static int hip_check(mns_handle* h, const char* what);

// cell count from which the automatic launch mode runs the mortar kernel on a
// second stream (measured on 3D Q2 meshes: slower at 32k cells, faster at
// 262k, 524k and 2M cells)
constexpr long long kConcurrentCells = 1 << 18;

// second stream (default priority) and fork/join events, created at setup
static int ensure_aux_stream(mns_handle* h) {
  if (h->aux && h->ev_fork && h->ev_join) return MNS_OK;
  return set_error(h, MNS_ERR_HIP, "second stream missing (handle not set up)");
}

static int hip_check(mns_handle* h, const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(h, MNS_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
  return MNS_OK;
}

// Launch of a kernel of timer class cls: while timing is enabled the launch
// carries the start and stop events of its own dispatch (so they bracket the
// kernel alone, not the queue around it).
template <typename K, typename... Args>
static void launch_k(mns_handle* h, int cls, K kernel, dim3 grid, dim3 block, hipStream_t s, Args... args) {
  if (h->timing_cap && h->ev_used[cls] < h->timing_cap) {
    const int u = h->ev_used[cls]++;
    hipExtLaunchKernelGGL(kernel, grid, block, 0, s, h->ev[cls][2 * u], h->ev[cls][2 * u + 1], 0, args...);
  } else {
    hipLaunchKernelGGL(kernel, grid, block, 0, s, args...);
  }
}

template <typename Real>
int launch_fill(Real* x, Real v, int64_t n, hipStream_t s) {
  if (n <= 0) return MNS_OK;
  long long blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_fill<Real>, dim3((unsigned)blocks), dim3(256), 0, s, x, v, (long long)n);
  return hipGetLastError() == hipSuccess ? MNS_OK : MNS_ERR_HIP;
}

template <typename Real>
int launch_constraints(const mns_handle* h, const Real* src, Real* dst, Real value, int mode, hipStream_t s) {
  if (h->n_cons == 0) return MNS_OK;
  const long long blocks = (h->n_cons + 255) / 256;
  hipLaunchKernelGGL(k_constraints<Real>, dim3((unsigned)blocks), dim3(256), 0, s, h->d_cons, (long long)h->n_cons,
                     src, dst, value, mode);
  return hipGetLastError() == hipSuccess ? MNS_OK : MNS_ERR_HIP;
}

#define MNS_DISPATCH(DIMV, KV, ...)                                 \
  switch (DIMV * 10 + KV) {                                          \
    case 22: { constexpr int DIM = 2, N = 3; __VA_ARGS__; } break;          \
    case 23: { constexpr int DIM = 2, N = 4; __VA_ARGS__; } break;          \
    case 24: { constexpr int DIM = 2, N = 5; __VA_ARGS__; } break;          \
    case 25: { constexpr int DIM = 2, N = 6; __VA_ARGS__; } break;          \
    case 32: { constexpr int DIM = 3, N = 3; __VA_ARGS__; } break;          \
    case 33: { constexpr int DIM = 3, N = 4; __VA_ARGS__; } break;          \
    case 34: { constexpr int DIM = 3, N = 5; __VA_ARGS__; } break;          \
    default: return set_error(h, MNS_ERR_UNSUPPORTED, "degree not compiled"); \
  }

template <typename Real, int DIM, int N>
static int do_mortar(mns_handle* h, const Real* src, Real* Em, int mask, hipStream_t s) {
  const Geom<Real> G = make_geom<Real>(h);
  const Tab1D<Real, N> T = make_tab<Real, N>(h);
  if (h->iso && h->equal_rings) {
    const auto* M = (const MortarTab<Real, N>*)(sizeof(Real) == 8 ? h->d_mtab64 : h->d_mtab32);
    const Real* mtrig = sizeof(Real) == 8 ? (const Real*)h->d_mtrig64 : (const Real*)h->d_mtrig32;
    const Real* img = sizeof(Real) == 8 ? (const Real*)h->d_mgeo64 : (const Real*)h->d_mgeo32;
    const unsigned blocks = (2u * (unsigned)(G.nth[0] * G.nz) + MortarShape<Real, DIM, N>::FPB - 1) /
                           MortarShape<Real, DIM, N>::FPB;
    launch_k(h, TIMER_MORTAR, k_mortar<Real, DIM, N, true>, dim3(blocks), dim3(64), s, G, T, h->k, M, mtrig, src, Em,
             mask, img);
    return hip_check(h, "iso-parametric mortar kernel");
  }
  if (h->iso) {
    const unsigned nfs = (unsigned)((h->nth[0] + h->nth[1]) * G.nz);
    MortarGen MG = make_mortar_gen(h);
    MG.iso_geo = sizeof(Real) == 8 ? (const void*)h->d_mgeo64 : (const void*)h->d_mgeo32;
    launch_k(h, TIMER_MORTAR, k_mortar_general<Real, DIM, N, true>, dim3(nfs), dim3(64), s, G, T, h->k, MG, src, Em,
             mask);
    return hip_check(h, "iso-parametric mortar kernel");
  }
  if (!h->equal_rings) {
    const unsigned nfs = (unsigned)((h->nth[0] + h->nth[1]) * G.nz);
    launch_k(h, TIMER_MORTAR, k_mortar_general<Real, DIM, N>, dim3(nfs), dim3(64), s, G, T, h->k, make_mortar_gen(h),
             src, Em, mask);
    return hip_check(h, "general mortar kernel");
  }
  const auto* M = (const MortarTab<Real, N>*)(sizeof(Real) == 8 ? h->d_mtab64 : h->d_mtab32);
  const Real* mtrig = sizeof(Real) == 8 ? (const Real*)h->d_mtrig64 : (const Real*)h->d_mtrig32;
  const unsigned blocks = (2u * (unsigned)(G.nth[0] * G.nz) + MortarShape<Real, DIM, N>::FPB - 1) /
                         MortarShape<Real, DIM, N>::FPB;
  launch_k(h, TIMER_MORTAR, k_mortar<Real, DIM, N>, dim3(blocks), dim3(64), s, G, T, h->k, M, mtrig, src, Em, mask,
           (const Real*)nullptr);
  return hip_check(h, "mortar kernel");
}

template <typename Real, int DIM, int N>
static int do_gather(mns_handle* h, const Real* E, const Real* Em, const Real* src, Real* dst, int mode,
                     hipStream_t s, int strip = 0) {
  const Geom<Real> G = make_geom<Real>(h);
  const long long nnodes = h->nnodes;
  launch_k(h, TIMER_OTHER, k_gather<Real, DIM, N>, dim3((unsigned)((nnodes + 255) / 256)), dim3(256), s, G, h->k, E,
           Em, src, dst, mode, strip);
  return hip_check(h, "gather kernel");
}

// the quad volume layout exists for 3D degrees 2 and 3 (degree 3 in FP64 at
// one wavefront per SIMD: its fused kernel holds about 480 registers per lane,
// and still runs 1.6x faster than the LDS-plane layout)
template <typename Real, int DIM, int N>
constexpr bool kQuadLayout = DIM == 3 && (N == 3 || N == 4);
// linearization source C in the quad kernels: FP32 at degrees 2 and 3, FP64
// at degree 2 (state point values in LDS next to the increment's, 32 KB per
// wavefront; at degree 3 they would need 57 KB)
template <typename Real, int DIM, int N>
constexpr bool kLinCLayout = kQuadLayout<Real, DIM, N> && (sizeof(Real) == 4 || N == 3);

template <typename Real, int DIM, int N>
static int do_jacobian(mns_handle* h, const Real* src, Real* dst, hipStream_t s, Real* E_ws = nullptr,
                       Real* Em_ws = nullptr) {
  using S = Shape<Real, DIM, N>;
  const Geom<Real> G = make_geom<Real>(h);
  const Tab1D<Real, N> T = make_tab<Real, N>(h);
  const Real* lin = sizeof(Real) == 8 ? (const Real*)h->d_lin64 : (const Real*)h->d_lin32;
  // local-result buffers: the handle's, or the caller's workspace
  Real* E = E_ws ? E_ws : (sizeof(Real) == 8 ? (Real*)h->d_E64 : (Real*)h->d_E32);
  Real* Em = Em_ws ? Em_ws : (sizeof(Real) == 8 ? (Real*)h->d_Em64 : (Real*)h->d_Em32);
  constexpr bool kQuad = kQuadLayout<Real, DIM, N>;
  // iso-parametric cells: LDS-plane layout with the per-point metric,
  // general mortar kernel in its own launch
  const bool iso = h->iso;
  const bool quad = kQuad && h->quad && !iso;
  // linearization source C (tau and tau R per point, a and grad u from the
  // state) where the quad kernels have it
  constexpr bool kLinC = kLinCLayout<Real, DIM, N>;
  const bool linc = kLinC && quad && h->lin_src[sizeof(Real) == 8 ? 0 : 1] == 1 && h->d_linc64;
  const Real* state = sizeof(Real) == 8 ? (const Real*)h->d_state : (const Real*)h->d_state32;
  if (linc) lin = sizeof(Real) == 8 ? (const Real*)h->d_linc64 : (const Real*)h->d_linc32;
  const int picard = h->lin_picard;
  // strip layout of the local results: batches of 16 cells stay inside one
  // ring when the ring length is a multiple of 16
  const int strip = (quad && h->nth[0] % 16 == 0 && h->nth[1] % 16 == 0) ? 1 : 0;
  const int cpw = quad ? QuadShape<Real, N>::CPW : S::CPW;
  const unsigned blocks = (unsigned)((G.ncells + cpw - 1) / cpw);
  int rc;
  // launch mode; automatic: one fused launch for small meshes (the mortar
  // work is a latency tail there), the concurrent second stream for large ones
  // (iso-parametric cells: the fused launch at every size, measured faster
  // than the second stream at 1.1M and 68M DoFs)
  int mode = h->fused >= 0 ? h->fused : (G.ncells >= kConcurrentCells && !iso ? 2 : 1);
  // unequal ring counts: the general mortar kernel runs as its own launch
  if (!h->equal_rings && mode == 1) mode = 0;
  if (mode == 1) {
    // one launch of volume cell blocks and mortar face blocks
    const auto* M = (const MortarTab<Real, N>*)(sizeof(Real) == 8 ? h->d_mtab64 : h->d_mtab32);
    const Real* mtrig = sizeof(Real) == 8 ? (const Real*)h->d_mtrig64 : (const Real*)h->d_mtrig32;
    const int nmb = (int)((2u * (unsigned)(G.nth[0] * G.nz) + MortarShape<Real, DIM, N>::FPB - 1) /
                          MortarShape<Real, DIM, N>::FPB);
    if constexpr (kQuad) {
      if (quad) {
        if constexpr (sizeof(Real) == 8 && N == 3) {
          using MSL = MortarShape<Real, DIM, N, kLdsQuadBytes>;
          const int nml = (int)((2u * (unsigned)(G.nth[0] * G.nz) + MSL::FPB - 1) / MSL::FPB);
          if (linc)
            launch_k(h, TIMER_VOLUME, k_jacobian_fused_quad_lds<N, true>, dim3(blocks + nml), dim3(64), s, G, T, h->k,
                     nml, lin, M, mtrig, src, E, Em, strip, state, picard);
          else
            launch_k(h, TIMER_VOLUME, k_jacobian_fused_quad_lds<N, false>, dim3(blocks + nml), dim3(64), s, G, T,
                     h->k, nml, lin, M, mtrig, src, E, Em, strip, state, picard);
        } else {
          if constexpr (kLinC) {
            if (linc)
              launch_k(h, TIMER_VOLUME, k_jacobian_fused_quad<Real, N, true>, dim3(blocks + nmb), dim3(64), s, G, T,
                       h->k, nmb, lin, M, mtrig, src, E, Em, strip, state, picard);
          }
          if (!linc)
            launch_k(h, TIMER_VOLUME, k_jacobian_fused_quad<Real, N, false>, dim3(blocks + nmb), dim3(64), s, G, T,
                     h->k, nmb, lin, M, mtrig, src, E, Em, strip, state, picard);
        }
      }
    }
    if (iso)
      launch_k(h, TIMER_VOLUME, k_jacobian_fused<Real, DIM, N, true>, dim3(blocks + nmb), dim3(64), s, G, T, h->k, nmb,
               lin, M, mtrig, src, E, Em,
               sizeof(Real) == 8 ? (const Real*)h->d_mgeo64 : (const Real*)h->d_mgeo32);
    else if (!quad)
      launch_k(h, TIMER_VOLUME, k_jacobian_fused<Real, DIM, N>, dim3(blocks + nmb), dim3(64), s, G, T, h->k, nmb, lin,
               M, mtrig, src, E, Em, (const Real*)nullptr);
    rc = hip_check(h, "fused volume/mortar kernel");
    if (rc) return rc;
  } else {
    // separate launches; with fused == 2 the mortar kernel runs on a second
    // stream next to the volume kernel (fork/join through events), so its
    // latency-bound wavefronts fill the volume kernel's idle issue slots
    const bool conc = mode == 2;
    hipStream_t ms = s;
    if (conc) {
      if ((rc = ensure_aux_stream(h))) return rc;
      ms = h->aux;
      if (hipEventRecord(h->ev_fork, s) != hipSuccess || hipStreamWaitEvent(ms, h->ev_fork, 0) != hipSuccess)
        return hip_check(h, "fork");
      rc = do_mortar<Real, DIM, N>(h, src, Em, 1, ms);
      if (rc) return rc;
    }
    if constexpr (kQuad) {
      if constexpr (kLinC) {
        if (linc)
          launch_k(h, TIMER_VOLUME, k_jacobian_volume_quad<Real, N, true>, dim3(blocks), dim3(64), s, G, T, h->k, lin,
                   src, E, strip, state, picard);
      }
      if (quad && !linc)
        launch_k(h, TIMER_VOLUME, k_jacobian_volume_quad<Real, N, false>, dim3(blocks), dim3(64), s, G, T, h->k, lin,
                 src, E, strip, state, picard);
    }
    if (iso)
      launch_k(h, TIMER_VOLUME, k_jacobian_volume<Real, DIM, N, true>, dim3(blocks), dim3(64), s, G, T, h->k, lin, src,
               E);
    else if (!quad)
      launch_k(h, TIMER_VOLUME, k_jacobian_volume<Real, DIM, N>, dim3(blocks), dim3(64), s, G, T, h->k, lin, src, E);
    rc = hip_check(h, "volume kernel");
    if (rc) return rc;
    if (conc) {
      if (hipEventRecord(h->ev_join, ms) != hipSuccess || hipStreamWaitEvent(s, h->ev_join, 0) != hipSuccess)
        return hip_check(h, "join");
    } else {
      rc = do_mortar<Real, DIM, N>(h, src, Em, 1, s);
      if (rc) return rc;
    }
  }
  return do_gather<Real, DIM, N>(h, E, Em, src, dst, 0, s, strip);
}

// ---------------------------------------------------------------------------
// Batched application: many instances of one dimension and degree in one
// volume + mortar launch and one gather launch.  One range of blocks
// integrates mortar faces, the other volume cells (which comes first follows
// the single-instance fused launch); the instance of a block is found by
// binary search in the block prefix sums.
// ---------------------------------------------------------------------------
__device__ inline int batch_item_of(const long long* __restrict__ start, int count, long long b) {
  int lo = 0, hi = count - 1;  // last instance whose range starts at or before b
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

template <typename Real, int N>
__global__ __launch_bounds__(64) void k_batch_jacobian_quad(const BatchItem<Real>* __restrict__ items,
                                                                          const long long* __restrict__ mstart,
                                                                          const long long* __restrict__ vstart,
                                                                          int count, Tab1D<Real, N> T, int k,
                                                                          const Real* __restrict__ src) {
  // FP64 degree 2: the layout of k_jacobian_fused_quad_lds (volume blocks
  // with their point values in LDS, two-face mortar blocks, one 18 KB buffer)
  constexpr bool kLds = sizeof(Real) == 8 && N == 3;
  constexpr int BUD = kLds ? kLdsQuadBytes : 36000;
  using MSm = MortarSmem<Real, 3, N, BUD>;
  constexpr int UB = kLds ? 4 * N * N * 64 * (int)sizeof(Real) : 0;
  constexpr int SB = (int)sizeof(MSm) > UB ? (int)sizeof(MSm) : UB;
  __shared__ __align__(16) unsigned char smem[SB];
  // volume blocks first, then the mortar blocks (degree 2; mortar first for
  // degree 3), as in the single-instance fused launches
  constexpr bool kVolumeFirst = N == 3;
  const long long mtot = mstart[count], vtot = vstart[count];
  const long long b = blockIdx.x;
  const bool mortar = kVolumeFirst ? b >= vtot : b < mtot;
  if (mortar) {
    const long long bm = kVolumeFirst ? b - vtot : b;
    const int i = batch_item_of(mstart, count, bm);
    const Geom<Real> G = items[i].G;
    mortar_block<Real, 3, N, BUD>(G, T, k, (int)(bm - mstart[i]), (const MortarTab<Real, N>*)items[i].mtab,
                                  items[i].mtrig, src + items[i].dof_off, items[i].Em, 1,
                                  *reinterpret_cast<MSm*>(smem));
  } else {
    const long long bv = kVolumeFirst ? b : b - mtot;
    const int i = batch_item_of(vstart, count, bv);
    const Geom<Real> G = items[i].G;
    volume_quad<Real, N, kLds>(G, T, k, (int)(bv - vstart[i]), items[i].lin, src + items[i].dof_off,
                               items[i].E, items[i].strip != 0, reinterpret_cast<Real*>(smem));
  }
}

// LDS-plane volume blocks and mortar blocks (2D, 3D degree 4, and curved
// cells of every degree: ISO, the blocks of the single-instance curved
// fused launch)
template <typename Real, int DIM, int N, bool ISO = false>
__global__ __launch_bounds__(64) void k_batch_jacobian(const BatchItem<Real>* __restrict__ items,
                                                                    const long long* __restrict__ mstart,
                                                                    const long long* __restrict__ vstart, int count,
                                                                    Tab1D<Real, N> T, int k,
                                                                    const Real* __restrict__ src) {
  __shared__ FusedSmem<Real, DIM, N, ISO> sm;
  const long long mtot = mstart[count];
  const long long b = blockIdx.x;
  if (b < mtot) {
    const int i = batch_item_of(mstart, count, b);
    const Geom<Real> G = items[i].G;
    mortar_block<Real, DIM, N, 36000, ISO>(G, T, k, (int)(b - mstart[i]), (const MortarTab<Real, N>*)items[i].mtab,
                                           items[i].mtrig, src + items[i].dof_off, items[i].Em, 1, sm.m,
                                           items[i].iso_mg);
  } else {
    const int i = batch_item_of(vstart, count, b - mtot);
    const Geom<Real> G = items[i].G;
    volume_block<Real, DIM, N, ISO>(G, T, k, (int)(b - mtot - vstart[i]), items[i].lin, src + items[i].dof_off,
                                    items[i].E, sm.v);
  }
}

template <typename Real, int DIM, int N>
__global__ __launch_bounds__(256) void k_batch_gather(const BatchItem<Real>* __restrict__ items,
                                                      const long long* __restrict__ gstart, int count, int k,
                                                      const Real* __restrict__ src, Real* __restrict__ dst) {
  const long long b = blockIdx.x;
  const int i = batch_item_of(gstart, count, b);
  const Geom<Real> G = items[i].G;
  const long long off = items[i].dof_off;
  gather_node<Real, DIM, N>(G, k, items[i].E, items[i].Em, src + off, dst + off, 0, items[i].strip,
                            (b - gstart[i]) * 256 + threadIdx.x);
}

// block counts of one instance in the batched launch (the layouts of
// do_jacobian's default configuration: quad volume layout where it exists)
template <typename Real, int DIM, int N>
static void batch_blocks(const mns_handle* h, long long* nmb, long long* nvb, int* strip) {
  using S = Shape<Real, DIM, N>;
  // curved cells: the LDS-plane layout of their fused launch
  const bool quad = kQuadLayout<Real, DIM, N> && !h->iso;
  const int cpw = quad ? QuadShape<Real, N>::CPW : S::CPW;
  *nvb = (h->ncells + cpw - 1) / cpw;
  // faces per mortar block: two in the FP64 degree-2 quad launch (its LDS is
  // shared with the LDS-staged volume blocks), the default otherwise
  const int FPB = (quad && sizeof(Real) == 8 && N == 3) ? MortarShape<Real, DIM, N, kLdsQuadBytes>::FPB
                                                        : MortarShape<Real, DIM, N>::FPB;
  *nmb = (2LL * h->nth[0] * h->nz + FPB - 1) / FPB;  // batches hold equal ring counts only
  *strip = (quad && h->nth[0] % 16 == 0) ? 1 : 0;
}

template <typename Real, int DIM, int N>
static void batch_items(const mns_batch* b, const mns_batch_group& g, std::vector<BatchItem<Real>>& items,
                        std::vector<long long>& ms, std::vector<long long>& vs) {
  const int count = (int)g.members.size();
  items.resize(count);
  ms.assign(count + 1, 0);
  vs.assign(count + 1, 0);
  for (int i = 0; i < count; ++i) {
    mns_handle* h = b->hs[g.members[i]];
    BatchItem<Real>& it = items[i];
    it.G = make_geom<Real>(h);
    it.lin = sizeof(Real) == 8 ? (const Real*)h->d_lin64 : (const Real*)h->d_lin32;
    it.E = sizeof(Real) == 8 ? (Real*)h->d_E64 : (Real*)h->d_E32;
    it.Em = sizeof(Real) == 8 ? (Real*)h->d_Em64 : (Real*)h->d_Em32;
    it.mtab = sizeof(Real) == 8 ? h->d_mtab64 : h->d_mtab32;
    it.mtrig = sizeof(Real) == 8 ? (const Real*)h->d_mtrig64 : (const Real*)h->d_mtrig32;
    it.dof_off = b->offsets[g.members[i]];  // offset in the whole batch's vectors
    it.iso_mg = h->iso ? (sizeof(Real) == 8 ? (const Real*)h->d_mgeo64 : (const Real*)h->d_mgeo32) : nullptr;
    long long nmb, nvb;
    batch_blocks<Real, DIM, N>(h, &nmb, &nvb, &it.strip);
    ms[i + 1] = ms[i] + nmb;
    vs[i + 1] = vs[i] + nvb;
  }
}

template <int DIM, int N>
static int batch_build_t(mns_batch* b, mns_batch_group& g) {
  std::vector<BatchItem<double>> i64;
  std::vector<BatchItem<float>> i32;
  std::vector<long long> ms64, vs64, ms32, vs32;
  batch_items<double, DIM, N>(b, g, i64, ms64, vs64);
  batch_items<float, DIM, N>(b, g, i32, ms32, vs32);
  const int count = (int)g.members.size();
  std::vector<long long> gs(count + 1, 0);
  for (int i = 0; i < count; ++i) gs[i + 1] = gs[i] + (b->hs[g.members[i]]->nnodes + 255) / 256;
  g.mtot[0] = ms64[count];
  g.vtot[0] = vs64[count];
  g.mtot[1] = ms32[count];
  g.vtot[1] = vs32[count];
  g.gtot = gs[count];
  std::vector<long long> prefix;
  for (const auto* v : {&ms64, &vs64, &ms32, &vs32, &gs}) prefix.insert(prefix.end(), v->begin(), v->end());
  hipError_t e;
  if ((e = hipMalloc(&g.d_items64, i64.size() * sizeof(i64[0]))) != hipSuccess ||
      (e = hipMalloc(&g.d_items32, i32.size() * sizeof(i32[0]))) != hipSuccess ||
      (e = hipMalloc((void**)&g.d_prefix, prefix.size() * sizeof(long long))) != hipSuccess ||
      (e = hipMemcpy(g.d_items64, i64.data(), i64.size() * sizeof(i64[0]), hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(g.d_items32, i32.data(), i32.size() * sizeof(i32[0]), hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(g.d_prefix, prefix.data(), prefix.size() * sizeof(long long), hipMemcpyHostToDevice)) !=
          hipSuccess) {
    b->err = std::string("batch tables: ") + hipGetErrorString(e);
    return MNS_ERR_HIP;
  }
  return MNS_OK;
}

int batch_build(mns_batch* b) {
  for (mns_batch_group& g : b->groups) {
    int rc;
    switch (g.dim * 10 + g.k) {
      case 22: rc = batch_build_t<2, 3>(b, g); break;
      case 23: rc = batch_build_t<2, 4>(b, g); break;
      case 24: rc = batch_build_t<2, 5>(b, g); break;
      case 25: rc = batch_build_t<2, 6>(b, g); break;
      case 32: rc = batch_build_t<3, 3>(b, g); break;
      case 33: rc = batch_build_t<3, 4>(b, g); break;
      case 34: rc = batch_build_t<3, 5>(b, g); break;
      default: b->err = "degree not compiled"; return MNS_ERR_UNSUPPORTED;
    }
    if (rc) return rc;
  }
  return MNS_OK;
}

// one group: its volume + mortar launch and its gather launch, on the whole
// batch's vectors (the items hold the instances' offsets)
template <typename Real, int DIM, int N>
static int do_batch(mns_batch* b, const mns_batch_group& g, const Real* src, Real* dst, hipStream_t s) {
  const int count = (int)g.members.size();
  const int p = sizeof(Real) == 8 ? 0 : 1;
  const auto* items = (const BatchItem<Real>*)(p == 0 ? g.d_items64 : g.d_items32);
  const long long* ms = g.d_prefix + (size_t)p * 2 * (count + 1);
  const long long* vs = ms + (count + 1);
  const long long* gs = g.d_prefix + (size_t)4 * (count + 1);
  const Tab1D<Real, N> T = make_tab<Real, N>(b->hs[g.members[0]]);
  const long long blocks = g.mtot[p] + g.vtot[p];
  constexpr bool kQuad = kQuadLayout<Real, DIM, N>;
  if (g.iso)
    hipLaunchKernelGGL((k_batch_jacobian<Real, DIM, N, true>), dim3((unsigned)blocks), dim3(64), 0, s, items, ms, vs,
                       count, T, g.k, src);
  else if constexpr (kQuad)
    hipLaunchKernelGGL((k_batch_jacobian_quad<Real, N>), dim3((unsigned)blocks), dim3(64), 0, s, items, ms, vs, count,
                       T, g.k, src);
  else
    hipLaunchKernelGGL((k_batch_jacobian<Real, DIM, N>), dim3((unsigned)blocks), dim3(64), 0, s, items, ms, vs,
                       count, T, g.k, src);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) {
    hipLaunchKernelGGL((k_batch_gather<Real, DIM, N>), dim3((unsigned)g.gtot), dim3(256), 0, s, items, gs, count,
                       g.k, src, dst);
    e = hipGetLastError();
  }
  if (e != hipSuccess) {
    b->err = std::string("batch kernels: ") + hipGetErrorString(e);
    return MNS_ERR_HIP;
  }
  return MNS_OK;
}

template <typename Real>
int launch_batch_jacobian(mns_batch* b, const Real* src, Real* dst, hipStream_t s) {
  for (const mns_batch_group& g : b->groups) {
    int rc;
    switch (g.dim * 10 + g.k) {
      case 22: rc = do_batch<Real, 2, 3>(b, g, src, dst, s); break;
      case 23: rc = do_batch<Real, 2, 4>(b, g, src, dst, s); break;
      case 24: rc = do_batch<Real, 2, 5>(b, g, src, dst, s); break;
      case 25: rc = do_batch<Real, 2, 6>(b, g, src, dst, s); break;
      case 32: rc = do_batch<Real, 3, 3>(b, g, src, dst, s); break;
      case 33: rc = do_batch<Real, 3, 4>(b, g, src, dst, s); break;
      case 34: rc = do_batch<Real, 3, 5>(b, g, src, dst, s); break;
      default: b->err = "degree not compiled"; return MNS_ERR_UNSUPPORTED;
    }
    if (rc) return rc;
  }
  return MNS_OK;
}
template int launch_batch_jacobian<double>(mns_batch*, const double*, double*, hipStream_t);
template int launch_batch_jacobian<float>(mns_batch*, const float*, float*, hipStream_t);

template <typename Real>
int launch_jacobian(mns_handle* h, const Real* src, Real* dst, hipStream_t s) {
  MNS_DISPATCH(h->dim, h->k, return (do_jacobian<Real, DIM, N>(h, src, dst, s)));
  return MNS_OK;
}

// ---------------------------------------------------------------------------
// Allocation-free Jacobian application.  The local-result buffers of the
// volume and mortar kernels (E, Em) come from one file-scope device array of
// kScratchBytes instead of the handle's buffers; every GPU that the library
// runs on holds its own copy until the process ends.  In host code the
// array's name is only a stand-in: its device address on the current device
// is looked up with hipGetSymbolAddress (once per device, at handle setup or
// on the entry point's first call there) and only that address is passed to
// kernels.  Nothing needs clearing between calls: every entry of E and Em
// that the gather reads is written by the same call.
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = size_t(32) << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

int scratch_pointer(void** out, size_t* bytes) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return MNS_ERR_HIP;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return MNS_ERR_HIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  if (bytes) *bytes = kScratchBytes;
  return MNS_OK;
}

// bytes of E and Em of one application in precision Real (E rounded up to
// 256 bytes so that Em starts aligned)
template <typename Real>
size_t jacobian_scratch_bytes(const mns_handle* h) {
  const size_t npt = (size_t)(h->dim == 3 ? h->n * h->n * h->n : h->n * h->n);
  const size_t e = ((size_t)h->ncells * h->nc * npt * sizeof(Real) + 255) / 256 * 256;
  const size_t em = (size_t)(h->nth[0] + h->nth[1]) * h->nz * h->nc * npt * sizeof(Real);
  return e + em;
}

template <typename Real>
int launch_jacobian_noalloc(mns_handle* h, const Real* src, Real* dst, hipStream_t s) {
  void* base = nullptr;
  size_t cap = 0;
  if (scratch_pointer(&base, &cap) != MNS_OK)
    return set_error(h, MNS_ERR_HIP, "device address of the scratch array not available");
  const size_t need = jacobian_scratch_bytes<Real>(h);
  if (need > cap)
    return set_error(h, MNS_ERR_UNSUPPORTED,
                     "mesh too large for the allocation-free apply: its local results need " + std::to_string(need) +
                         " bytes, the scratch array holds " + std::to_string(cap));
  const size_t npt = (size_t)(h->dim == 3 ? h->n * h->n * h->n : h->n * h->n);
  Real* E = (Real*)base;
  Real* Em = (Real*)((unsigned char*)base + ((size_t)h->ncells * h->nc * npt * sizeof(Real) + 255) / 256 * 256);
  MNS_DISPATCH(h->dim, h->k, return (do_jacobian<Real, DIM, N>(h, src, dst, s, E, Em)));
  return MNS_OK;
}
template int launch_jacobian_noalloc<double>(mns_handle*, const double*, double*, hipStream_t);
template int launch_jacobian_noalloc<float>(mns_handle*, const float*, float*, hipStream_t);

// tau and tau R of every point (linearization source C) from the full store,
// in FP64 and FP32
__global__ void k_lin_compact(const double* __restrict__ lin, long long npts, double* __restrict__ c64,
                              float* __restrict__ c32) {
  using LL = LinLayout<3>;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < npts; p += stride) {
    const double* l = lin + p * LL::SIZE;
    const double v[4] = {l[LL::TAU], l[LL::TR], l[LL::TR + 1], l[LL::TR + 2]};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      c64[p * 4 + j] = v[j];
      c32[p * 4 + j] = (float)v[j];
    }
  }
}

int launch_lin_compact(mns_handle* h, hipStream_t s) {
  if (!h->d_linc64) return MNS_OK;
  const long long npts = (long long)h->ncells * h->n * h->n * h->n;
  long long b = (npts + 255) / 256;
  if (b > 8192) b = 8192;
  hipLaunchKernelGGL(k_lin_compact, dim3((unsigned)b), dim3(256), 0, s, (const double*)h->d_lin64, npts, h->d_linc64,
                     h->d_linc32);
  return hip_check(h, "linearization C kernel");
}

template <int DIM, int N, bool RES>
static int do_state(mns_handle* h, const double* state, const double* hist, const double* force, double* lin,
                    double* res, hipStream_t s) {
  using S = Shape<double, DIM, N>;
  const Geom<double> G = make_geom<double>(h);
  const Tab1D<double, N> T = make_tab<double, N>(h);
  const unsigned blocks = (unsigned)((G.ncells + S::CPW - 1) / S::CPW);
  if (h->iso)
    hipLaunchKernelGGL((k_state_iso<DIM, N, RES>), dim3(blocks), dim3(64), 0, s, G, T, h->k, state, hist, force, lin,
                       res, RES ? 0 : h->picard);
  else
    hipLaunchKernelGGL((k_state<DIM, N, RES>), dim3(blocks), dim3(64), 0, s, G, T, h->k, state, hist, force, lin,
                       res, RES ? 0 : h->picard);
  return hip_check(h, RES ? "residual kernel" : "linearization kernel");
}

template <>
int launch_linearize<double>(mns_handle* h, const double* state, const double* hist, const double* force,
                             double* lin, hipStream_t s) {
  MNS_DISPATCH(h->dim, h->k, return (do_state<DIM, N, false>(h, state, hist, force, lin, nullptr, s)));
  return MNS_OK;
}

int launch_residual(mns_handle* h, const double* state, double* res, hipStream_t s) {
  int rc = MNS_OK;
  MNS_DISPATCH(h->dim, h->k, {
    rc = do_state<DIM, N, true>(h, state, h->desc.steady ? nullptr : h->d_hist, h->d_force, nullptr, h->d_E64, s);
    if (rc) return rc;
    rc = do_mortar<double, DIM, N>(h, state, h->d_Em64, 0, s);
    if (rc) return rc;
    rc = do_gather<double, DIM, N>(h, h->d_E64, h->d_Em64, state, res, 1, s);
    if (rc) return rc;
  });
  return MNS_OK;
}

// segment slots per face side: a face meets at most ceil(ratio) + 1 faces of
// the other ring, ratio the larger of the two cell-angle ratios
int iso_mortar_pieces(const mns_handle* h) {
  const int a = std::max(h->nth[0], h->nth[1]), b = std::min(h->nth[0], h->nth[1]);
  return std::min(kMaxPieces, (a + b - 1) / b + 1);
}

int launch_iso_mortar_geo(mns_handle* h, hipStream_t s) {
  if (!h->iso) return MNS_OK;
  const unsigned nfs = (unsigned)((h->nth[0] + h->nth[1]) * h->nz);
  MNS_DISPATCH(h->dim, h->k, {
    hipLaunchKernelGGL((k_iso_mortar_geo<DIM, N>), dim3(nfs), dim3(64), 0, s, make_geom<double>(h),
                       make_tab<double, N>(h), h->k, make_mortar_gen(h), h->equal_rings ? 1 : 0, h->m,
                       h->phi / h->dthd[1], h->d_mgeo64, h->d_mgeo32);
  });
  return hip_check(h, "iso-parametric mortar geometry kernel");
}

template <typename Real, int DIM, int N>
static int do_diag(mns_handle* h, Real* diag, hipStream_t s) {
  using S = Shape<Real, DIM, N>;
  const Geom<Real> G = make_geom<Real>(h);
  const Tab1D<Real, N> T = make_tab<Real, N>(h);
  const Real* lin = sizeof(Real) == 8 ? (const Real*)h->d_lin64 : (const Real*)h->d_lin32;
  int rc = launch_fill<Real>(diag, Real(0), h->ndofs, s);
  if (rc) return set_error(h, rc, "fill");
  const long long total = (long long)G.ncells * S::NPT;
  if (h->iso)
    hipLaunchKernelGGL((k_diag_volume<Real, DIM, N, true>), dim3((unsigned)((total + 127) / 128)), dim3(128), 0, s, G,
                       T, h->k, lin, diag);
  else
    hipLaunchKernelGGL((k_diag_volume<Real, DIM, N>), dim3((unsigned)((total + 127) / 128)), dim3(128), 0, s, G, T,
                       h->k, lin, diag);
  rc = hip_check(h, "diagonal kernel");
  if (rc) return rc;
  if (h->iso) {
    hipLaunchKernelGGL((k_mortar_diag_iso<Real, DIM, N>), dim3((unsigned)((h->nth[0] + h->nth[1]) * G.nz)), dim3(64),
                       0, s, G, T, h->k, make_mortar_gen(h), diag);
  } else if (h->equal_rings) {
    const auto* M = (const MortarTab<Real, N>*)(sizeof(Real) == 8 ? h->d_mtab64 : h->d_mtab32);
    const Real* mtrig = sizeof(Real) == 8 ? (const Real*)h->d_mtrig64 : (const Real*)h->d_mtrig32;
    hipLaunchKernelGGL((k_mortar_diag<Real, DIM, N>), dim3(2u * (unsigned)(G.nth[0] * G.nz)), dim3(64), 0, s, G, T,
                       h->k, M, mtrig, diag);
  } else {
    hipLaunchKernelGGL((k_mortar_diag_general<Real, DIM, N>), dim3((unsigned)((h->nth[0] + h->nth[1]) * G.nz)),
                       dim3(64), 0, s, G, T, h->k, make_mortar_gen(h), diag);
  }
  rc = hip_check(h, "mortar diagonal kernel");
  if (rc) return rc;
  rc = launch_constraints<Real>(h, diag, diag, Real(1), 2, s);
  return rc ? set_error(h, rc, "constraints") : MNS_OK;
}

template <typename Real>
int launch_diagonal(mns_handle* h, Real* diag, hipStream_t s) {
  MNS_DISPATCH(h->dim, h->k, return (do_diag<Real, DIM, N>(h, diag, s)));
  return MNS_OK;
}

template int launch_jacobian<double>(mns_handle*, const double*, double*, hipStream_t);
template int launch_jacobian<float>(mns_handle*, const float*, float*, hipStream_t);
template int launch_diagonal<double>(mns_handle*, double*, hipStream_t);
template int launch_diagonal<float>(mns_handle*, float*, hipStream_t);
template int launch_fill<double>(double*, double, int64_t, hipStream_t);
template int launch_fill<float>(float*, float, int64_t, hipStream_t);
template int launch_constraints<double>(const mns_handle*, const double*, double*, double, int, hipStream_t);
template int launch_constraints<float>(const mns_handle*, const float*, float*, float, int, hipStream_t);

}  // namespace mns
