// Device-side indexing of the structured rotor/stator meshes shared by the
// kernel sources: per-cell work shape, cell decoding and the global node of a
// cell's local node.
#pragma once

#include "mns_internal.hpp"

namespace mns {

template <typename Real, int DIM, int N>
struct Shape {
  static constexpr int NZ = (DIM == 3) ? N : 1;  // line length along z
  static constexpr int PLANE = N * N;
  static constexpr int TPC = N * N;              // lanes per cell
  static constexpr int CPW = 64 / TPC;           // cells per wavefront
  static constexpr int NPT = PLANE * NZ;         // nodes (= quadrature points) per cell
  static constexpr int NC = DIM + 1;             // components
  static constexpr int NYV = (DIM == 3) ? 5 : 3; // r-stage outputs per velocity component
  static constexpr int NYP = (DIM == 3) ? 3 : 2; // r-stage outputs of the pressure
  static constexpr int NT = DIM + 1;             // test coefficients per component
  static constexpr int EVAL_SLOTS = DIM * NYV + NYP;
  static constexpr int TEST_SLOTS = NC * NT;
  static constexpr int SLOTS = (EVAL_SLOTS > TEST_SLOTS) ? EVAL_SLOTS : TEST_SLOTS;
  // LDS layout of the per-cell work arrays: cell c owns [c * REGION, ...),
  // element stride ES = 1
  static constexpr int ES = 1;
  static constexpr int REGION = SLOTS * NPT;
  template <int NSLOTS>
  static constexpr int lds_size() {
    return (CPW - 1) * (NSLOTS * NPT) + NSLOTS * NPT;
  }
};

struct CellId {
  int dom, ct, cr, cz;
};

// per-domain parameter selected without indexing the kernel-argument block
// by a lane-dependent value (which would turn into a vector memory load)
template <typename T>
__device__ inline T pick(int d, const T (&a)[2]) {
  return d ? a[1] : a[0];
}

template <typename Real>
__device__ inline CellId decode_cell(const Geom<Real>& G, int cell) {
  CellId c;
  c.dom = cell >= (int)G.cell_off1;
  int l = cell - (c.dom ? (int)G.cell_off1 : 0);
  const int nt = pick(c.dom, G.nth);
  c.ct = l % nt;
  l /= nt;
  const int nr = pick(c.dom, G.nr);
  c.cr = l % nr;
  c.cz = l / nr;
  return c;
}

// global node of local node (a, b, c) of cell C; also returns the node's
// structured indices for the constraint predicates
template <typename Real, int DIM>
__device__ inline long long node_of(const Geom<Real>& G, int k, const CellId& C, int a, int b, int c, int& it,
                                    int& ir, int& iz) {
  it = k * C.ct + a;
  const int ntn = pick(C.dom, G.ntd);
  if (it >= ntn) it -= ntn;
  ir = k * C.cr + b;
  iz = (DIM == 3) ? k * C.cz + c : 0;
  long long base = C.dom ? G.node_off1 : 0;
  return base + it + (long long)ntn * (ir + (long long)pick(C.dom, G.nrn) * iz);
}

}  // namespace mns
