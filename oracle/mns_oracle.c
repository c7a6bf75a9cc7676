/*
 * mns_oracle.c -- plain FP64 CPU oracle for the linearized SUPG/PSPG-stabilized
 * ALE Navier-Stokes operator on a rotor/stator pair of annular Q_k meshes
 * coupled by mortar face integrals.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this library.  It shares no code,
 * header, table or helper with the HIP library; the product path never calls it.
 *
 * What it computes (all in double precision, element by element, with full
 * tensor-product basis tables and no sum factorization):
 *   - weak form with mortar terms: Sec. 2 and 2.1, Eqs. EqNSweak, EqMortarPre,
 *     EqMortarDiff, EqPenalty, EqMortarMass, Eq-NSweakWmortar;
 *   - SUPG/PSPG stabilization and Tezduyar tau: Sec. 2.2, Eqs.
 *     Eq-NSweakComplete, Eq-strong-residual, Eq-stab-param;
 *   - Newton Jacobian blocks: Sec. 2.3, Eqs. Eq-Newton-method, Eq-Newton-matrix
 *     and the stabilized/Galerkin block definitions (Eq-discrete-1..4); as an
 *     option (picard = 1) the same blocks with the derivative of the
 *     convection velocity and of the SUPG weight left out (the Oseen operator
 *     that the multigrid preconditioner approximates);
 *   - rigid rotor rotation x = R x0: Sec. 3.1;
 *   - mortar segments with one reference quadrature mapped into each segment and
 *     det J = R * (segment angle) * (layer height): Sec. 3.2, Eq. Eq-Jacobian;
 *   - diagonal by unit-vector columns (Alg. Alg-diagonal) and the assembled
 *     matrix (Alg. Alg-matrix) for tiny meshes;
 *   - the 2D manufactured solution of Sec. 4.1 (forcing and L2 errors).
 *
 * Readings taken where the paper is silent or garbled (the same list is kept in
 * the design notes):
 *   - jump and normal are taken per side: jump = own - other, n = own outward
 *     normal (rotor +e_r, stator -e_r); this is textbook SIPG with n = n^-;
 *   - the SUPG weight derivative is tau (du . grad v) . R and the B-hat SUPG
 *     term is (tau (a . grad) v, grad dp); tau is frozen in the Jacobian;
 *   - penalty F default 1; rule 0 uses each side's own cell tau_k, rule 1 the
 *     max of both sides; "interior" faces are all non-mortar faces;
 *   - the mortar Jacobian uses the segment ANGLE: JxW = w_q R dtheta_seg dz;
 *   - h = 2 sqrt(A/pi) in 2D and (6V/pi)^(1/3) in 3D;
 *   - exact polar geometry, GLL nodes, n = k+1 Gauss points per direction;
 *   - no-slip on all external walls, one pressure DoF pinned.
 *
 * Layout: DoF = node*(d+1) + comp, comps (ux, uy[, uz], p).  Per domain nodes
 * are lexicographic with theta fastest (periodic, k*n_theta positions), then r
 * (k*n_r+1), then z (k*n_z+1).  Rotor block first.  Rotor nodes are numbered in
 * the rotor's material frame.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define MAXN 7
#define MAXND (MAXN * MAXN * MAXN)

typedef struct {
  int dim, degree;
  double r_in, r_if, r_out, height;
  int n_theta, n_r_rotor, n_r_stator, n_z;
  double nu, penalty_F;
  int penalty_rule;
  int steady;
  double dt;
  double theta_rot, omega;
  int merged;        /* 1: one conforming mesh, interface nodes shared, no mortar */
  int stabilization; /* 1: SUPG + PSPG terms on */
  int pin_pressure;  /* 1: pin one pressure DoF */
  int mms;           /* 1: analytic forcing of the 2D manufactured solution */
  int nthreads;
  int picard;        /* 1: Jacobian of the Picard (Oseen) linearization: the
                        convection velocity and the SUPG weight are frozen at
                        the state, so the reaction term (du . grad) u and the
                        SUPG weight derivative are absent */
  int n_theta_stator; /* cells per ring of the stator; 0: n_theta (the equal
                         interface counts of Sec. 2.1 / Sec. 3.1).  Unequal
                         counts are the extension named in Sec. 3.1 and Sec. 5:
                         a face may then meet more than two faces of the other
                         side, every intersection being one mortar segment */
  int iso;           /* 1: iso-parametric geometry (the Q_k mapping the paper's
                        meshes use, Sec. 2.1): every cell is the Q_k
                        interpolant of its node positions, which are the polar
                        Gauss-Lobatto nodes moved by the interior perturbation
                        below; 0: the exact polar map */
  double perturb;    /* iso = 1: amplitude of the node perturbation in cell
                        sizes (radial, angular and axial displacements that
                        vanish on the walls and on the interface, so that these
                        stay circles / planes through their nodes); a mesh
                        whose map folds (det J zero or of the wrong sign at a
                        Gauss-Lobatto point of a cell) is refused: a Q2 mid
                        node moved by a quarter cell already makes the map
                        singular on a face */
} orc_params;

/* ------------------------------------------------------------------------ */
/* 1D rules                                                                  */
/* ------------------------------------------------------------------------ */

/* Legendre P_m(x) and P_m'(x) by the three-term recurrence. */
static void legendre(int m, double x, double *P, double *dP) {
  double p0 = 1.0, p1 = x;
  if (m == 0) { *P = 1.0; *dP = 0.0; return; }
  for (int j = 2; j <= m; ++j) {
    double p2 = ((2.0 * j - 1.0) * x * p1 - (j - 1.0) * p0) / j;
    p0 = p1; p1 = p2;
  }
  *P = p1;
  /* P_m' = m (x P_m - P_{m-1}) / (x^2 - 1) away from +-1 */
  *dP = m * (x * p1 - p0) / (x * x - 1.0);
}

/* n-point Gauss-Legendre rule mapped to [0,1]. */
static void gauss01(int n, double *x, double *w) {
  for (int i = 0; i < n; ++i) {
    double t = cos(M_PI * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double P, dP;
      legendre(n, t, &P, &dP);
      double dt = P / dP;
      t -= dt;
      if (fabs(dt) < 1e-16) break;
    }
    double P, dP;
    legendre(n, t, &P, &dP);
    double wt = 2.0 / ((1.0 - t * t) * dP * dP);
    x[n - 1 - i] = 0.5 * (1.0 + t);
    w[n - 1 - i] = 0.5 * wt;
  }
}

/* n-point Gauss-Lobatto nodes on [0,1]: endpoints plus the roots of P_{n-1}'. */
static void lobatto01(int n, double *x) {
  int N = n - 1;
  x[0] = 0.0;
  x[N] = 1.0;
  for (int i = 1; i < N; ++i) {
    /* roots of P_N' via Newton on q(t) = P_N'(t); q' from the Legendre ODE */
    double t = -cos(M_PI * i / N);
    for (int it = 0; it < 100; ++it) {
      double P, dP;
      legendre(N, t, &P, &dP);
      double d2P = (2.0 * t * dP - N * (N + 1.0) * P) / (1.0 - t * t);
      double dt = dP / d2P;
      t -= dt;
      if (fabs(dt) < 1e-16) break;
    }
    x[i] = 0.5 * (1.0 + t);
  }
}

/* Lagrange basis on nodes xn[0..n-1]: values, first and second derivatives at t,
 * each written straight from the product definition. */
static void lagrange(int n, const double *xn, double t, double *L, double *dL, double *d2L) {
  for (int j = 0; j < n; ++j) {
    double v = 1.0;
    for (int m = 0; m < n; ++m)
      if (m != j) v *= (t - xn[m]) / (xn[j] - xn[m]);
    L[j] = v;
    double d1 = 0.0;
    for (int l = 0; l < n; ++l) {
      if (l == j) continue;
      double prod = 1.0 / (xn[j] - xn[l]);
      for (int m = 0; m < n; ++m)
        if (m != j && m != l) prod *= (t - xn[m]) / (xn[j] - xn[m]);
      d1 += prod;
    }
    dL[j] = d1;
    double d2 = 0.0;
    for (int l = 0; l < n; ++l) {
      if (l == j) continue;
      for (int k = 0; k < n; ++k) {
        if (k == j || k == l) continue;
        double prod = 1.0 / ((xn[j] - xn[l]) * (xn[j] - xn[k]));
        for (int m = 0; m < n; ++m)
          if (m != j && m != l && m != k) prod *= (t - xn[m]) / (xn[j] - xn[m]);
        d2 += prod;
      }
    }
    d2L[j] = d2;
  }
}

/* ------------------------------------------------------------------------ */
/* Mesh                                                                      */
/* ------------------------------------------------------------------------ */

typedef struct {
  int dom;       /* storage domain */
  int rotor;     /* 1: rotor material (ALE velocity omega e_z x x) */
  int ct, cr, cz;
  double th0, dth, r0, dr, z0, dz;
  int iface;     /* 1: one face lies on the mortar interface */
  double h;      /* element size for tau_u */
  double tau_pen;/* Hillewaert penalty of this cell (interface cells) */
} cell_t;

typedef struct {
  int cz, ct_rotor, ct_stator;
  double lo, hi; /* physical angles of the segment */
} seg_t;

typedef struct {
  orc_params P;
  int d, k, n, nd, nc;
  int ndom;
  int nr[2];
  int nth[2];          /* cells per ring of each storage domain */
  int ntd[2];          /* theta node positions per ring of each domain */
  int ntn, nrn[2], nzn;
  long noff[2];
  long nnodes, ndofs;
  double dth, dz;      /* dth: cell angle of the rotor (domain 0) */
  double dthd[2];      /* cell angle of each domain */
  double gll[MAXN], gx[MAXN], gw[MAXN];
  long ncell_dom[2], coff[2], ncells;
  cell_t *cells;
  long nseg;
  seg_t *segs;
  unsigned char *cons; /* constrained DoF flags */
  double tau_side[2];  /* penalty used by side 0 (rotor) and 1 (stator) */
  double *xnode;       /* iso: physical node positions [node][3] (rotor rotated) */
} mesh_t;

static void cell_radial(const mesh_t *M, int dom, int cr, double *r0, double *dr, int *rotor) {
  const orc_params *P = &M->P;
  if (!P->merged) {
    if (dom == 0) {
      *dr = (P->r_if - P->r_in) / P->n_r_rotor;
      *r0 = P->r_in + cr * (*dr);
      *rotor = 1;
    } else {
      *dr = (P->r_out - P->r_if) / P->n_r_stator;
      *r0 = P->r_if + cr * (*dr);
      *rotor = 0;
    }
  } else {
    if (cr < P->n_r_rotor) {
      *dr = (P->r_if - P->r_in) / P->n_r_rotor;
      *r0 = P->r_in + cr * (*dr);
      *rotor = 1;
    } else {
      *dr = (P->r_out - P->r_if) / P->n_r_stator;
      *r0 = P->r_if + (cr - P->n_r_rotor) * (*dr);
      *rotor = 0;
    }
  }
}

/* global node id of local node (a0,a1,a2) of cell c */
static long cell_node(const mesh_t *M, const cell_t *c, int a0, int a1, int a2) {
  const long ntn = M->ntd[c->dom];
  long it = (M->k * (long)c->ct + a0) % ntn;
  long ir = M->k * (long)c->cr + a1;
  long iz = (M->d == 3) ? (M->k * (long)c->cz + a2) : 0;
  return M->noff[c->dom] + it + ntn * (ir + (long)M->nrn[c->dom] * iz);
}

static void local_idx(const mesh_t *M, int a, int *a0, int *a1, int *a2) {
  *a0 = a % M->n;
  *a1 = (a / M->n) % M->n;
  *a2 = (M->d == 3) ? a / (M->n * M->n) : 0;
}

static void cell_dofs(const mesh_t *M, const cell_t *c, long *dofs) {
  for (int a = 0; a < M->nd; ++a) {
    int a0, a1, a2;
    local_idx(M, a, &a0, &a1, &a2);
    long node = cell_node(M, c, a0, a1, a2);
    for (int comp = 0; comp < M->nc; ++comp) dofs[a * M->nc + comp] = node * M->nc + comp;
  }
}

/* ------------------------------------------------------------------------ */
/* Geometry: exact polar (cylindrical) map                                   */
/*   theta = th0 + dth xi0,  r = r0 + dr xi1,  z = z0 + dz xi2               */
/*   x = r cos theta, y = r sin theta, z                                     */
/* ------------------------------------------------------------------------ */

static void geom_iso(const mesh_t *M, const cell_t *c, const double xi[3], double x[3], double J[3][3],
                     double X2[3][3][3]);

static void geom(const mesh_t *M, const cell_t *c, const double xi[3], double x[3], double J[3][3],
                 double X2[3][3][3]) {
  if (M->xnode) {
    geom_iso(M, c, xi, x, J, X2);
    return;
  }
  double th = c->th0 + c->dth * xi[0];
  double r = c->r0 + c->dr * xi[1];
  double ct = cos(th), st = sin(th);
  memset(J, 0, sizeof(double) * 9);
  memset(X2, 0, sizeof(double) * 27);
  x[0] = r * ct;
  x[1] = r * st;
  x[2] = (M->d == 3) ? c->z0 + c->dz * xi[2] : 0.0;
  /* J[m][a] = d x_m / d xi_a */
  J[0][0] = -r * st * c->dth;
  J[1][0] = r * ct * c->dth;
  J[0][1] = ct * c->dr;
  J[1][1] = st * c->dr;
  if (M->d == 3) J[2][2] = c->dz;
  /* X2[m][a][b] = d^2 x_m / d xi_a d xi_b */
  X2[0][0][0] = -r * ct * c->dth * c->dth;
  X2[1][0][0] = -r * st * c->dth * c->dth;
  X2[0][0][1] = X2[0][1][0] = -st * c->dth * c->dr;
  X2[1][0][1] = X2[1][1][0] = ct * c->dth * c->dr;
}

/* ------------------------------------------------------------------------ */
/* Geometry: iso-parametric Q_k map (orc_params.iso)                         */
/*   x(xi) = sum_a X_a phi_a(xi), X_a the cell's node positions, phi_a the    */
/*   tensor Lagrange basis on the Gauss-Lobatto nodes; J and the Hessian of   */
/*   the map follow from the basis derivatives.                               */
/* ------------------------------------------------------------------------ */

static void geom_iso(const mesh_t *M, const cell_t *c, const double xi[3], double x[3], double J[3][3],
                     double X2[3][3][3]) {
  const int n = M->n, d = M->d;
  double L[3][MAXN], dL[3][MAXN], d2L[3][MAXN];
  for (int dir = 0; dir < 3; ++dir)
    if (dir < d) lagrange(n, M->gll, xi[dir], L[dir], dL[dir], d2L[dir]);
  memset(x, 0, sizeof(double) * 3);
  memset(J, 0, sizeof(double) * 9);
  memset(X2, 0, sizeof(double) * 27);
  for (int a = 0; a < M->nd; ++a) {
    int ai[3];
    local_idx(M, a, &ai[0], &ai[1], &ai[2]);
    const double *X = M->xnode + 3 * cell_node(M, c, ai[0], ai[1], ai[2]);
    double val = 1.0, g[3] = {0, 0, 0}, H[3][3] = {{0}};
    for (int dir = 0; dir < d; ++dir) val *= L[dir][ai[dir]];
    for (int p = 0; p < d; ++p) {
      double v = 1.0;
      for (int dir = 0; dir < d; ++dir) v *= (dir == p) ? dL[dir][ai[dir]] : L[dir][ai[dir]];
      g[p] = v;
      for (int q = 0; q < d; ++q) {
        double h = 1.0;
        for (int dir = 0; dir < d; ++dir) {
          if (p == q && dir == p) h *= d2L[dir][ai[dir]];
          else if (dir == p || dir == q) h *= dL[dir][ai[dir]];
          else h *= L[dir][ai[dir]];
        }
        H[p][q] = h;
      }
    }
    for (int m = 0; m < d; ++m) {
      x[m] += X[m] * val;
      for (int p = 0; p < d; ++p) {
        J[m][p] += X[m] * g[p];
        for (int q = 0; q < d; ++q) X2[m][p][q] += X[m] * H[p][q];
      }
    }
  }
}

/* Physical position of local node (a0, a1, a2) of cell c for the
 * iso-parametric mesh: the polar Gauss-Lobatto node (r, theta, z), moved in
 * the material frame by
 *   dr     = e dr_c  s(r) cos(3 theta_m + 2 pi z / H)
 *   dtheta = e dth_c s(r) sin(2 theta_m) (1 + cos(2 pi z / H) / 2)
 *   dz     = e dz    s(r) sin(theta_m) sin(pi z / H)           (3D)
 * with theta_m the material angle and s(r) = sin(pi (r - r_a) / (r_b - r_a))
 * on the node's domain [r_a, r_b] (rotor [r_in, R], stator [R, r_out]), so
 * that walls, interface and the planes z = 0, H keep their nodes; rotor
 * nodes are then rotated by theta_rot (x = R(theta) x0, Sec. 3.1). */
static void node_position(const mesh_t *M, const cell_t *c, int a0, int a1, int a2, double X[3]) {
  const orc_params *P = &M->P;
  const double e = P->perturb;
  const double rot = (!P->merged && c->dom == 0) ? P->theta_rot : 0.0;
  const double thm = c->th0 - rot + c->dth * M->gll[a0];
  const double r = c->r0 + c->dr * M->gll[a1];
  const double z = (M->d == 3) ? c->z0 + c->dz * M->gll[a2] : 0.0;
  const double H = (M->d == 3) ? P->height : 1.0;
  const int rotor_side = r < P->r_if || (r == P->r_if && c->rotor);
  const double ra = rotor_side ? P->r_in : P->r_if, rb = rotor_side ? P->r_if : P->r_out;
  const double s = sin(M_PI * (r - ra) / (rb - ra));
  const double zr = (M->d == 3) ? 2.0 * M_PI * z / H : 0.0;
  const double dr = e * c->dr * s * cos(3.0 * thm + zr);
  const double dt = e * c->dth * s * sin(2.0 * thm) * (1.0 + 0.5 * cos(zr));
  const double dz = (M->d == 3) ? e * c->dz * s * sin(thm) * sin(M_PI * z / H) : 0.0;
  const double rr = r + dr, th = thm + dt + rot;
  X[0] = rr * cos(th);
  X[1] = rr * sin(th);
  X[2] = z + dz;
}

static double inverse(int d, double J[3][3], double Ji[3][3]) {
  double det;
  memset(Ji, 0, sizeof(double) * 9);
  if (d == 2) {
    det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    Ji[0][0] = J[1][1] / det;
    Ji[0][1] = -J[0][1] / det;
    Ji[1][0] = -J[1][0] / det;
    Ji[1][1] = J[0][0] / det;
  } else {
    det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
          J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    Ji[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
    Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
    Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
    Ji[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
    Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
    Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
    Ji[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
    Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
    Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
  }
  return det;
}

/* Physical basis: values, gradients and Laplacians of all n^d local shape
 * functions at reference point xi, through the generic chain rule
 *   grad phi = J^{-T} grad_xi phi,
 *   Hess phi = J^{-T} (Hess_xi phi - sum_m (grad phi)_m Hess_xi x_m) J^{-1}. */
typedef struct {
  double phi[MAXND], g[MAXND][3], lap[MAXND];
  double x[3];
  double detJ;
} pbasis_t;

static void phys_basis(const mesh_t *M, const cell_t *c, const double xi[3], pbasis_t *B) {
  int n = M->n, d = M->d;
  double L[3][MAXN], dL[3][MAXN], d2L[3][MAXN];
  for (int dir = 0; dir < d; ++dir) lagrange(n, M->gll, xi[dir], L[dir], dL[dir], d2L[dir]);
  double J[3][3], X2[3][3][3], Ji[3][3];
  geom(M, c, xi, B->x, J, X2);
  B->detJ = inverse(d, J, Ji);
  for (int a = 0; a < M->nd; ++a) {
    int ai[3];
    local_idx(M, a, &ai[0], &ai[1], &ai[2]);
    double gr[3] = {0, 0, 0}, H[3][3] = {{0}};
    double val = 1.0;
    for (int dir = 0; dir < d; ++dir) val *= L[dir][ai[dir]];
    for (int p = 0; p < d; ++p) {
      double v = 1.0;
      for (int dir = 0; dir < d; ++dir) v *= (dir == p) ? dL[dir][ai[dir]] : L[dir][ai[dir]];
      gr[p] = v;
      for (int q = 0; q < d; ++q) {
        double h = 1.0;
        for (int dir = 0; dir < d; ++dir) {
          if (p == q && dir == p) h *= d2L[dir][ai[dir]];
          else if (dir == p || dir == q) h *= dL[dir][ai[dir]];
          else h *= L[dir][ai[dir]];
        }
        H[p][q] = h;
      }
    }
    B->phi[a] = val;
    double gp[3] = {0, 0, 0};
    for (int m = 0; m < d; ++m)
      for (int p = 0; p < d; ++p) gp[m] += Ji[p][m] * gr[p];
    for (int m = 0; m < 3; ++m) B->g[a][m] = (m < d) ? gp[m] : 0.0;
    double Mh[3][3];
    for (int p = 0; p < d; ++p)
      for (int q = 0; q < d; ++q) {
        double s = H[p][q];
        for (int m = 0; m < d; ++m) s -= gp[m] * X2[m][p][q];
        Mh[p][q] = s;
      }
    double lap = 0.0;
    for (int m = 0; m < d; ++m) {
      double hmm = 0.0;
      for (int p = 0; p < d; ++p)
        for (int q = 0; q < d; ++q) hmm += Ji[p][m] * Mh[p][q] * Ji[q][m];
      lap += hmm;
    }
    B->lap[a] = lap;
  }
}

/* measures by quadrature of the exact map */
static double cell_measure(const mesh_t *M, const cell_t *c) {
  double V = 0.0;
  int n = M->n, nq = (M->d == 3) ? n * n * n : n * n;
  for (int q = 0; q < nq; ++q) {
    double xi[3] = {M->gx[q % n], M->gx[(q / n) % n], (M->d == 3) ? M->gx[q / (n * n)] : 0.0};
    double w = M->gw[q % n] * M->gw[(q / n) % n] * ((M->d == 3) ? M->gw[q / (n * n)] : 1.0);
    double x[3], J[3][3], X2[3][3][3], Ji[3][3];
    geom(M, c, xi, x, J, X2);
    V += w * fabs(inverse(M->d, J, Ji));
  }
  return V;
}

/* area (3D) or length (2D) of the face where reference coordinate `dir` = `val` */
static double face_measure(const mesh_t *M, const cell_t *c, int dir, double val) {
  int n = M->n, d = M->d;
  double A = 0.0;
  int other[2], no = 0;
  for (int e = 0; e < d; ++e)
    if (e != dir) other[no++] = e;
  int nq = (d == 3) ? n * n : n;
  for (int q = 0; q < nq; ++q) {
    double xi[3] = {0, 0, 0};
    xi[dir] = val;
    xi[other[0]] = M->gx[q % n];
    double w = M->gw[q % n];
    if (d == 3) { xi[other[1]] = M->gx[q / n]; w *= M->gw[q / n]; }
    double x[3], J[3][3], X2[3][3][3];
    geom(M, c, xi, x, J, X2);
    double t0[3] = {J[0][other[0]], J[1][other[0]], J[2][other[0]]};
    if (d == 2) {
      A += w * sqrt(t0[0] * t0[0] + t0[1] * t0[1]);
    } else {
      double t1[3] = {J[0][other[1]], J[1][other[1]], J[2][other[1]]};
      double cx = t0[1] * t1[2] - t0[2] * t1[1];
      double cy = t0[2] * t1[0] - t0[0] * t1[2];
      double cz = t0[0] * t1[1] - t0[1] * t1[0];
      A += w * sqrt(cx * cx + cy * cy + cz * cz);
    }
  }
  return A;
}

static int mesh_build(const orc_params *P, mesh_t *M) {
  memset(M, 0, sizeof(*M));
  M->P = *P;
  if (P->dim != 2 && P->dim != 3) return -1;
  if (P->degree < 1 || P->degree + 1 > MAXN) return -1;
  if (P->dim == 3 && P->degree + 1 > 6) return -1;
  if (!(P->r_in > 0 && P->r_in < P->r_if && P->r_if < P->r_out)) return -1;
  if (P->n_theta < 3 || P->n_r_rotor < 1 || P->n_r_stator < 1) return -1;
  if (P->dim == 3 && (P->n_z < 1 || !(P->height > 0))) return -1;
  if (P->merged && P->theta_rot != 0.0) return -1;
  if (P->n_theta_stator != 0 && (P->n_theta_stator < 3 || (P->merged && P->n_theta_stator != P->n_theta))) return -1;
  M->d = P->dim;
  M->k = P->degree;
  M->n = P->degree + 1;
  M->nd = (M->d == 3) ? M->n * M->n * M->n : M->n * M->n;
  M->nc = M->d + 1;
  M->ndom = P->merged ? 1 : 2;
  if (P->merged) {
    M->nr[0] = P->n_r_rotor + P->n_r_stator;
  } else {
    M->nr[0] = P->n_r_rotor;
    M->nr[1] = P->n_r_stator;
  }
  int nz = (M->d == 3) ? P->n_z : 1;
  M->ntn = M->k * P->n_theta;
  M->nzn = (M->d == 3) ? M->k * nz + 1 : 1;
  M->dth = 2.0 * M_PI / P->n_theta;
  M->nth[0] = P->n_theta;
  M->nth[1] = P->n_theta_stator > 0 ? P->n_theta_stator : P->n_theta;
  for (int dm = 0; dm < 2; ++dm) {
    M->ntd[dm] = M->k * M->nth[dm];
    M->dthd[dm] = 2.0 * M_PI / M->nth[dm];
  }
  M->dz = (M->d == 3) ? P->height / nz : 1.0;
  lobatto01(M->n, M->gll);
  gauss01(M->n, M->gx, M->gw);
  long off = 0, coff = 0;
  for (int dm = 0; dm < M->ndom; ++dm) {
    M->nrn[dm] = M->k * M->nr[dm] + 1;
    M->noff[dm] = off;
    off += (long)M->ntd[dm] * M->nrn[dm] * M->nzn;
    M->ncell_dom[dm] = (long)M->nth[dm] * M->nr[dm] * nz;
    M->coff[dm] = coff;
    coff += M->ncell_dom[dm];
  }
  M->nnodes = off;
  M->ndofs = off * M->nc;
  M->ncells = coff;
  M->cells = (cell_t *)calloc((size_t)M->ncells, sizeof(cell_t));
  if (!M->cells) return -2;
  for (int dm = 0; dm < M->ndom; ++dm)
    for (int cz = 0; cz < nz; ++cz)
      for (int cr = 0; cr < M->nr[dm]; ++cr)
        for (int ct = 0; ct < M->nth[dm]; ++ct) {
          cell_t *c = &M->cells[M->coff[dm] + ct + (long)M->nth[dm] * (cr + (long)M->nr[dm] * cz)];
          c->dom = dm;
          c->ct = ct;
          c->cr = cr;
          c->cz = cz;
          cell_radial(M, dm, cr, &c->r0, &c->dr, &c->rotor);
          c->dth = M->dthd[dm];
          /* x = R(theta_rot) x0 on every rotor node (Sec. 3.1) */
          c->th0 = ct * c->dth + ((!P->merged && dm == 0) ? P->theta_rot : 0.0);
          c->z0 = cz * M->dz;
          c->dz = M->dz;
          c->iface = !P->merged && ((dm == 0 && cr == M->nr[0] - 1) || (dm == 1 && cr == 0));
        }
  if (P->iso) {
    /* node positions of the iso-parametric mesh (each node written by every
     * cell that holds it, with the same value up to rounding) */
    M->xnode = (double *)calloc((size_t)M->nnodes * 3, sizeof(double));
    if (!M->xnode) return -2;
    for (long ci = 0; ci < M->ncells; ++ci) {
      const cell_t *c = &M->cells[ci];
      for (int a = 0; a < M->nd; ++a) {
        int a0, a1, a2;
        local_idx(M, a, &a0, &a1, &a2);
        node_position(M, c, a0, a1, a2, M->xnode + 3 * cell_node(M, c, a0, a1, a2));
      }
    }
  }
  for (int dm = 0; dm < M->ndom; ++dm)
    for (int cz = 0; cz < nz; ++cz)
      for (int cr = 0; cr < M->nr[dm]; ++cr)
        for (int ct = 0; ct < M->nth[dm]; ++ct) {
          cell_t *c = &M->cells[M->coff[dm] + ct + (long)M->nth[dm] * (cr + (long)M->nr[dm] * cz)];
          if (M->xnode) {
            /* an iso-parametric cell must map one-to-one: det J keeps the sign
             * of the polar map at every Gauss-Lobatto point (faces and corners
             * included); the reference axes (theta, r, z) are left-handed, so
             * that sign is negative */
            for (int a = 0; a < M->nd; ++a) {
              int a0, a1, a2;
              local_idx(M, a, &a0, &a1, &a2);
              double xi[3] = {M->gll[a0], M->gll[a1], M->gll[a2]}, x[3], J[3][3], X2[3][3][3], Ji[3][3];
              geom(M, c, xi, x, J, X2);
              if (!(inverse(M->d, J, Ji) < 0.0)) return -4;
            }
          }
          double V = cell_measure(M, c);
          c->h = (M->d == 2) ? 2.0 * sqrt(V / M_PI) : cbrt(6.0 * V / M_PI);
          if (c->iface) {
            /* Eq. EqPenalty: F (k+1)^2 [A(non-mortar faces)/2 + A(mortar face)] / V */
            double Am = face_measure(M, c, 1, dm == 0 ? 1.0 : 0.0);
            double Ao = face_measure(M, c, 1, dm == 0 ? 0.0 : 1.0) + face_measure(M, c, 0, 0.0) +
                        face_measure(M, c, 0, 1.0);
            if (M->d == 3) Ao += face_measure(M, c, 2, 0.0) + face_measure(M, c, 2, 1.0);
            c->tau_pen = P->penalty_F * (M->k + 1.0) * (M->k + 1.0) * (0.5 * Ao + Am) / V;
          }
        }
  if (!P->merged) {
    /* all rotor interface cells share one tau, all stator interface cells another */
    M->tau_side[0] = M->cells[M->coff[0] + (long)M->nth[0] * (M->nr[0] - 1)].tau_pen;
    M->tau_side[1] = M->cells[M->coff[1]].tau_pen;
    if (P->penalty_rule == 1) {
      double t = fmax(M->tau_side[0], M->tau_side[1]);
      M->tau_side[0] = M->tau_side[1] = t;
    }
    /* mortar segments: intersect every stator interface face with every rotor
     * interface face on the circle (Sec. 2.1, Sec. 3.2) */
    long cap = 4L * (M->nth[0] + M->nth[1]) * nz + 8;
    M->segs = (seg_t *)calloc((size_t)cap, sizeof(seg_t));
    if (!M->segs) return -2;
    long ns = 0;
    const double dts = M->dthd[1], dtr = M->dthd[0], tol = 1e-12 * fmin(dts, dtr);
    for (int cz = 0; cz < nz; ++cz)
      for (int js = 0; js < M->nth[1]; ++js) {
        double lo_s = js * dts, hi_s = lo_s + dts;
        for (int ir = 0; ir < M->nth[0]; ++ir) {
          double lo_r0 = P->theta_rot + ir * dtr;
          for (int sh = -3; sh <= 3; ++sh) {
            double lo_r = lo_r0 + 2.0 * M_PI * sh, hi_r = lo_r + dtr;
            double lo = fmax(lo_s, lo_r), hi = fmin(hi_s, hi_r);
            if (hi - lo > tol) {
              if (ns >= cap) return -3;
              M->segs[ns].cz = cz;
              M->segs[ns].ct_rotor = ir;
              M->segs[ns].ct_stator = js;
              M->segs[ns].lo = lo;
              M->segs[ns].hi = hi;
              ++ns;
            }
          }
        }
      }
    M->nseg = ns;
  }
  /* constraints: no-slip velocity on every external wall, one pressure pin */
  M->cons = (unsigned char *)calloc((size_t)M->ndofs, 1);
  if (!M->cons) return -2;
  for (int dm = 0; dm < M->ndom; ++dm)
    for (long iz = 0; iz < M->nzn; ++iz)
      for (long ir = 0; ir < M->nrn[dm]; ++ir)
        for (long it = 0; it < M->ntd[dm]; ++it) {
          long node = M->noff[dm] + it + M->ntd[dm] * (ir + M->nrn[dm] * iz);
          int wall = 0;
          if (ir == 0 && (P->merged || dm == 0)) wall = 1;                 /* r = r_in */
          if (ir == M->nrn[dm] - 1 && (P->merged || dm == 1)) wall = 1;    /* r = r_out */
          if (M->d == 3 && (iz == 0 || iz == M->nzn - 1)) wall = 1;        /* z = 0, H */
          if (wall)
            for (int comp = 0; comp < M->d; ++comp) M->cons[node * M->nc + comp] = 1;
        }
  if (P->pin_pressure) {
    int dm = M->ndom - 1;
    long node = M->noff[dm] + 0 + M->ntd[dm] * (M->nrn[dm] - 1);
    M->cons[node * M->nc + M->d] = 1;
  }
  return 0;
}

static void mesh_free(mesh_t *M) {
  free(M->cells);
  free(M->segs);
  free(M->cons);
  free(M->xnode);
}

/* ------------------------------------------------------------------------ */
/* Pointwise physics                                                         */
/* ------------------------------------------------------------------------ */

typedef struct {
  double u[3], gu[3][3], lu[3], p, gp[3]; /* gu[m][n] = d u_m / d x_n */
} field_t;

static void eval_field(const mesh_t *M, const pbasis_t *B, const double *loc, field_t *F) {
  int d = M->d, nc = M->nc;
  memset(F, 0, sizeof(*F));
  for (int a = 0; a < M->nd; ++a) {
    for (int m = 0; m < d; ++m) {
      double v = loc[a * nc + m];
      F->u[m] += B->phi[a] * v;
      for (int e = 0; e < d; ++e) F->gu[m][e] += B->g[a][e] * v;
      F->lu[m] += B->lap[a] * v;
    }
    double pv = loc[a * nc + d];
    F->p += B->phi[a] * pv;
    for (int e = 0; e < d; ++e) F->gp[e] += B->g[a][e] * pv;
  }
}

/* Tezduyar stabilization parameter, Eq. Eq-stab-param */
static double tau_u(const mesh_t *M, const double a[3], double h) {
  double an2 = 0.0;
  for (int m = 0; m < M->d; ++m) an2 += a[m] * a[m];
  double ct = M->P.steady ? 0.0 : 1.0 / M->P.dt;
  double nu = M->P.nu;
  double s = ct * ct + 4.0 * an2 / (h * h) + 9.0 * (4.0 * nu / (h * h)) * (4.0 * nu / (h * h));
  return (s > 0.0) ? 1.0 / sqrt(s) : 0.0;
}

static double time_coef(const mesh_t *M) { return M->P.steady ? 0.0 : 1.5 / M->P.dt; }

/* 2D manufactured solution of Sec. 4.1 and its derivatives */
static void mms_fields(const double x[3], double u[3], double gu[3][3], double lu[3], double *p, double gp[3]) {
  double a = M_PI * x[0], b = M_PI * x[1];
  double sa = sin(a), ca = cos(a), sb = sin(b), cb = cos(b);
  double s2a = sin(2 * a), c2a = cos(2 * a), s2b = sin(2 * b), c2b = cos(2 * b);
  double pi = M_PI, pi2 = M_PI * M_PI;
  memset(gu, 0, sizeof(double) * 9);
  u[0] = -2.0 * sa * sa * cb * sb;
  u[1] = 2.0 * ca * sa * sb * sb;
  u[2] = 0.0;
  gu[0][0] = -pi * s2a * s2b;
  gu[0][1] = -2.0 * pi * sa * sa * c2b;
  gu[1][0] = 2.0 * pi * c2a * sb * sb;
  gu[1][1] = pi * s2a * s2b;
  lu[0] = -2.0 * pi2 * c2a * s2b + 4.0 * pi2 * sa * sa * s2b;
  lu[1] = -4.0 * pi2 * s2a * sb * sb + 2.0 * pi2 * s2a * c2b;
  lu[2] = 0.0;
  *p = sa * sb;
  gp[0] = pi * ca * sb;
  gp[1] = pi * sa * cb;
  gp[2] = 0.0;
}

/* steady forcing that makes the manufactured field exact for the ALE momentum
 * equation: f = ((u - w) . grad) u + grad p - nu lap u */
static void mms_forcing(const mesh_t *M, const double x[3], const double w[3], double f[3]) {
  double u[3], gu[3][3], lu[3], p, gp[3];
  mms_fields(x, u, gu, lu, &p, gp);
  for (int m = 0; m < 3; ++m) {
    double conv = 0.0;
    for (int e = 0; e < 2; ++e) conv += gu[m][e] * (u[e] - w[e]);
    f[m] = (m < 2) ? conv + gp[m] - M->P.nu * lu[m] : 0.0;
  }
}

typedef struct {
  double gv[3], Gv[3][3], gq, Gq[3];
} testcoef_t;

/* strong momentum residual at the state, Eq. Eq-strong-residual (BDF2 history
 * hist, forcing f) */
static void strong_residual(const mesh_t *M, const field_t *S, const double hist[3], const double f[3],
                            const double a[3], double R[3]) {
  double ct = time_coef(M);
  for (int m = 0; m < M->d; ++m) {
    double conv = 0.0;
    for (int e = 0; e < M->d; ++e) conv += S->gu[m][e] * a[e];
    R[m] = ct * S->u[m] + hist[m] + conv + S->gp[m] - M->P.nu * S->lu[m] - f[m];
  }
  for (int m = M->d; m < 3; ++m) R[m] = 0.0;
}

/* Linearized volume integrand at one point: the stabilized blocks A-hat,
 * B-hat, C-hat, D-hat applied to the increment T. */
static void pw_jacobian(const mesh_t *M, const field_t *S, const double hist[3], const double f[3],
                        const double w[3], double tau, const field_t *T, testcoef_t *C) {
  int d = M->d;
  double nu = M->P.nu, ct = time_coef(M);
  int stab = M->P.stabilization;
  double a[3] = {0, 0, 0}, R[3], Rp[3] = {0, 0, 0};
  for (int m = 0; m < d; ++m) a[m] = S->u[m] - w[m];
  strong_residual(M, S, hist, f, a, R);
  memset(C, 0, sizeof(*C));
  for (int m = 0; m < d; ++m) {
    double reac = 0.0, conv = 0.0;
    for (int e = 0; e < d; ++e) {
      reac += S->gu[m][e] * T->u[e];
      conv += T->gu[m][e] * a[e];
    }
    if (M->P.picard) reac = 0.0;
    C->gv[m] = ct * T->u[m] + reac + conv;
    Rp[m] = ct * T->u[m] + reac + conv - nu * T->lu[m] + T->gp[m];
  }
  if (M->P.picard)
    for (int m = 0; m < d; ++m) R[m] = 0.0; /* no SUPG weight derivative */
  for (int m = 0; m < d; ++m)
    for (int e = 0; e < d; ++e) {
      C->Gv[m][e] = nu * T->gu[m][e] - (m == e ? T->p : 0.0);
      if (stab) C->Gv[m][e] += tau * Rp[m] * a[e] + tau * R[m] * T->u[e];
    }
  C->gq = 0.0;
  for (int m = 0; m < d; ++m) C->gq += T->gu[m][m];
  for (int m = 0; m < d; ++m) C->Gq[m] = stab ? tau * Rp[m] : 0.0;
}

/* Nonlinear volume integrand (residual) at the state S; tau given. */
static void pw_residual(const mesh_t *M, const field_t *S, const double hist[3], const double f[3],
                        const double w[3], double tau, testcoef_t *C) {
  int d = M->d;
  double nu = M->P.nu, ct = time_coef(M);
  int stab = M->P.stabilization;
  double a[3] = {0, 0, 0}, R[3];
  for (int m = 0; m < d; ++m) a[m] = S->u[m] - w[m];
  strong_residual(M, S, hist, f, a, R);
  memset(C, 0, sizeof(*C));
  for (int m = 0; m < d; ++m) {
    double conv = 0.0;
    for (int e = 0; e < d; ++e) conv += S->gu[m][e] * a[e];
    C->gv[m] = ct * S->u[m] + hist[m] + conv - f[m];
  }
  for (int m = 0; m < d; ++m)
    for (int e = 0; e < d; ++e) {
      C->Gv[m][e] = nu * S->gu[m][e] - (m == e ? S->p : 0.0);
      if (stab) C->Gv[m][e] += tau * R[m] * a[e];
    }
  C->gq = 0.0;
  for (int m = 0; m < d; ++m) C->gq += S->gu[m][m];
  for (int m = 0; m < d; ++m) C->Gq[m] = stab ? tau * R[m] : 0.0;
}

/* test function a, component comp, against the coefficients */
static double test_dot(const mesh_t *M, const pbasis_t *B, int a, int comp, const testcoef_t *C) {
  int d = M->d;
  double s;
  if (comp < d) {
    s = B->phi[a] * C->gv[comp];
    for (int e = 0; e < d; ++e) s += B->g[a][e] * C->Gv[comp][e];
  } else {
    s = B->phi[a] * C->gq;
    for (int e = 0; e < d; ++e) s += B->g[a][e] * C->Gq[e];
  }
  return s;
}

static void ale_velocity(const mesh_t *M, const cell_t *c, const double x[3], double w[3]) {
  w[0] = w[1] = w[2] = 0.0;
  if (c->rotor) {
    w[0] = -M->P.omega * x[1];
    w[1] = M->P.omega * x[0];
  }
}

/* reference quadrature point q of a cell */
static double cell_qp(const mesh_t *M, int q, double xi[3]) {
  int n = M->n;
  xi[0] = M->gx[q % n];
  xi[1] = M->gx[(q / n) % n];
  xi[2] = (M->d == 3) ? M->gx[q / (n * n)] : 0.0;
  return M->gw[q % n] * M->gw[(q / n) % n] * ((M->d == 3) ? M->gw[q / (n * n)] : 1.0);
}

static void gather(const mesh_t *M, const long *dofs, const double *vec, int mask_cons, double *loc) {
  int ndl = M->nd * M->nc;
  for (int i = 0; i < ndl; ++i) {
    if (!vec) { loc[i] = 0.0; continue; }
    loc[i] = (mask_cons && M->cons[dofs[i]]) ? 0.0 : vec[dofs[i]];
  }
}

/* vector value of a nodal field at a point (first d components) */
static void interp_vec(const mesh_t *M, const pbasis_t *B, const double *loc, double out[3]) {
  out[0] = out[1] = out[2] = 0.0;
  if (!loc) return;
  for (int a = 0; a < M->nd; ++a)
    for (int m = 0; m < M->d; ++m) out[m] += B->phi[a] * loc[a * M->nc + m];
}

/* ------------------------------------------------------------------------ */
/* Volume loops                                                              */
/* ------------------------------------------------------------------------ */

enum { MODE_JAC = 0, MODE_RES = 1, MODE_DIAG = 2 };

typedef struct {
  const double *state, *hist, *force, *x, *tau_state;
} inputs_t;

/* per-cell work: local output (nd*nc) */
static void cell_volume(const mesh_t *M, const cell_t *c, const inputs_t *in, int mode, double *yloc) {
  int ndl = M->nd * M->nc;
  long dofs[MAXND * 4];
  double Sl[MAXND * 4], Xl[MAXND * 4], Hl[MAXND * 4], Fl[MAXND * 4], Tl[MAXND * 4];
  cell_dofs(M, c, dofs);
  gather(M, dofs, in->state, 0, Sl);
  gather(M, dofs, in->hist, 0, Hl);
  gather(M, dofs, in->force, 0, Fl);
  if (mode == MODE_JAC) gather(M, dofs, in->x, 1, Xl);
  if (in->tau_state) gather(M, dofs, in->tau_state, 0, Tl);
  memset(yloc, 0, sizeof(double) * ndl);
  pbasis_t *B = (pbasis_t *)malloc(sizeof(pbasis_t));
  int nq = M->nd;
  for (int q = 0; q < nq; ++q) {
    double xi[3];
    double wq = cell_qp(M, q, xi);
    phys_basis(M, c, xi, B);
    double JxW = wq * fabs(B->detJ);
    field_t S;
    eval_field(M, B, Sl, &S);
    double w[3], hist[3], f[3];
    ale_velocity(M, c, B->x, w);
    interp_vec(M, B, (in->hist && !M->P.steady) ? Hl : NULL, hist);
    if (M->P.mms) mms_forcing(M, B->x, w, f);
    else interp_vec(M, B, in->force ? Fl : NULL, f);
    double a[3] = {0, 0, 0};
    if (in->tau_state) {
      field_t Ts;
      eval_field(M, B, Tl, &Ts);
      for (int m = 0; m < M->d; ++m) a[m] = Ts.u[m] - w[m];
    } else {
      for (int m = 0; m < M->d; ++m) a[m] = S.u[m] - w[m];
    }
    double tau = tau_u(M, a, c->h);
    testcoef_t C;
    if (mode == MODE_JAC) {
      field_t T;
      eval_field(M, B, Xl, &T);
      pw_jacobian(M, &S, hist, f, w, tau, &T, &C);
      for (int i = 0; i < ndl; ++i) yloc[i] += JxW * test_dot(M, B, i / M->nc, i % M->nc, &C);
    } else if (mode == MODE_RES) {
      pw_residual(M, &S, hist, f, w, tau, &C);
      for (int i = 0; i < ndl; ++i) yloc[i] += JxW * test_dot(M, B, i / M->nc, i % M->nc, &C);
    } else {
      /* diagonal: column i of the element matrix, entry i (Alg. Alg-diagonal for
       * the volume part) */
      for (int i = 0; i < ndl; ++i) {
        int a_ = i / M->nc, comp = i % M->nc;
        field_t T;
        memset(&T, 0, sizeof(T));
        if (comp < M->d) {
          T.u[comp] = B->phi[a_];
          for (int e = 0; e < M->d; ++e) T.gu[comp][e] = B->g[a_][e];
          T.lu[comp] = B->lap[a_];
        } else {
          T.p = B->phi[a_];
          for (int e = 0; e < M->d; ++e) T.gp[e] = B->g[a_][e];
        }
        pw_jacobian(M, &S, hist, f, w, tau, &T, &C);
        yloc[i] += JxW * test_dot(M, B, a_, comp, &C);
      }
    }
  }
  free(B);
}

static int color_of(const mesh_t *M, const cell_t *c) {
  return (c->ct & 1) + 2 * (c->cr & 1) + 4 * (c->cz & 1);
}

static void volume_loop(const mesh_t *M, const inputs_t *in, int mode, const unsigned char *cell_mask, double *y) {
  int ndl = M->nd * M->nc;
  int par = (M->nth[0] % 2 == 0) && (M->nth[1] % 2 == 0) && M->P.nthreads != 1;
#ifdef _OPENMP
  if (M->P.nthreads > 0) omp_set_num_threads(M->P.nthreads);
#endif
  if (par) {
    for (int color = 0; color < 8; ++color) {
#pragma omp parallel
      {
        double *yloc = (double *)malloc(sizeof(double) * ndl);
        long dofs[MAXND * 4];
#pragma omp for schedule(dynamic, 16)
        for (long ci = 0; ci < M->ncells; ++ci) {
          const cell_t *c = &M->cells[ci];
          if (color_of(M, c) != color) continue;
          if (cell_mask && !cell_mask[ci]) continue;
          cell_volume(M, c, in, mode, yloc);
          cell_dofs(M, c, dofs);
          for (int i = 0; i < ndl; ++i) y[dofs[i]] += yloc[i];
        }
        free(yloc);
      }
    }
  } else {
    double *yloc = (double *)malloc(sizeof(double) * ndl);
    long dofs[MAXND * 4];
    for (long ci = 0; ci < M->ncells; ++ci) {
      const cell_t *c = &M->cells[ci];
      if (cell_mask && !cell_mask[ci]) continue;
      cell_volume(M, c, in, mode, yloc);
      cell_dofs(M, c, dofs);
      for (int i = 0; i < ndl; ++i) y[dofs[i]] += yloc[i];
    }
    free(yloc);
  }
}

/* ------------------------------------------------------------------------ */
/* Mortar                                                                     */
/* ------------------------------------------------------------------------ */

static const cell_t *iface_cell(const mesh_t *M, int side, int ct, int cz) {
  int cr = (side == 0) ? M->nr[0] - 1 : 0;
  return &M->cells[M->coff[side] + ct + (long)M->nth[side] * (cr + (long)M->nr[side] * cz)];
}

/* reference coordinates on `side` of the physical mortar point (theta, z) */
static void mortar_xi(const mesh_t *M, const cell_t *c, int side, double th, double xiz, double xi[3]) {
  double t = fmod(th - c->th0, 2.0 * M_PI);
  if (t < 0) t += 2.0 * M_PI;
  if (t > 2.0 * M_PI - 0.5 * c->dth) t -= 2.0 * M_PI;
  xi[0] = t / c->dth;
  xi[1] = (side == 0) ? 1.0 : 0.0;
  xi[2] = xiz;
}

/* side-s face coefficients of Eqs. EqMortarPre, EqMortarDiff, EqMortarMass:
 * v_s  <- {p} n_s - nu {grad u} n_s + nu tau_s j_s
 * grad v_s <- -(nu/2) j_s (x) n_s
 * q_s  <- -(1/2) j_s . n_s
 * with j_s = u_s - u_o and n_s the outward normal of side s. */
static void mortar_coef(const mesh_t *M, int side, const field_t *Fs, const field_t *Fo, const double ns[3],
                        testcoef_t *C) {
  int d = M->d;
  double nu = M->P.nu, tau = M->tau_side[side];
  double j[3] = {0, 0, 0};
  for (int m = 0; m < d; ++m) j[m] = Fs->u[m] - Fo->u[m];
  double pbar = 0.5 * (Fs->p + Fo->p);
  memset(C, 0, sizeof(*C));
  for (int m = 0; m < d; ++m) {
    double gn = 0.0;
    for (int e = 0; e < d; ++e) gn += 0.5 * (Fs->gu[m][e] + Fo->gu[m][e]) * ns[e];
    C->gv[m] = pbar * ns[m] - nu * gn + nu * tau * j[m];
    for (int e = 0; e < d; ++e) C->Gv[m][e] = -0.5 * nu * j[m] * ns[e];
  }
  double jn = 0.0;
  for (int m = 0; m < d; ++m) jn += j[m] * ns[m];
  C->gq = -0.5 * jn;
}

/* Mortar face terms applied to nodal vector xv (already masked), added to y.
 * Each segment carries a Gauss rule in theta (and in z) mapped into it. */
static void mortar_loop(const mesh_t *M, const double *xv, const unsigned char *cell_mask, double *y) {
  if (M->P.merged) return;
  int n = M->n, d = M->d, nc = M->nc, ndl = M->nd * nc;
  int nqz = (d == 3) ? n : 1;
  pbasis_t *B[2];
  B[0] = (pbasis_t *)malloc(sizeof(pbasis_t));
  B[1] = (pbasis_t *)malloc(sizeof(pbasis_t));
  double *yl[2];
  yl[0] = (double *)malloc(sizeof(double) * ndl);
  yl[1] = (double *)malloc(sizeof(double) * ndl);
  for (long s = 0; s < M->nseg; ++s) {
    const seg_t *sg = &M->segs[s];
    const cell_t *c[2] = {iface_cell(M, 0, sg->ct_rotor, sg->cz), iface_cell(M, 1, sg->ct_stator, sg->cz)};
    long ci0 = c[0] - M->cells, ci1 = c[1] - M->cells;
    int want[2] = {!cell_mask || cell_mask[ci0], !cell_mask || cell_mask[ci1]};
    if (!want[0] && !want[1]) continue;
    long dofs[2][MAXND * 4];
    double Xl[2][MAXND * 4];
    for (int sd = 0; sd < 2; ++sd) {
      cell_dofs(M, c[sd], dofs[sd]);
      for (int i = 0; i < ndl; ++i) Xl[sd][i] = xv[dofs[sd][i]];
      memset(yl[sd], 0, sizeof(double) * ndl);
    }
    double len = sg->hi - sg->lo;
    for (int qz = 0; qz < nqz; ++qz)
      for (int qt = 0; qt < n; ++qt) {
        double th = sg->lo + M->gx[qt] * len;
        double xiz = (d == 3) ? M->gx[qz] : 0.0;
        /* Eq. Eq-Jacobian with the segment angle: w R dtheta_seg dz */
        double JxW = M->gw[qt] * M->P.r_if * len * ((d == 3) ? M->gw[qz] * M->dz : 1.0);
        field_t F[2];
        for (int sd = 0; sd < 2; ++sd) {
          double xi[3];
          mortar_xi(M, c[sd], sd, th, xiz, xi);
          phys_basis(M, c[sd], xi, B[sd]);
          eval_field(M, B[sd], Xl[sd], &F[sd]);
        }
        double er[3] = {cos(th), sin(th), 0.0};
        for (int sd = 0; sd < 2; ++sd) {
          if (!want[sd]) continue;
          double ns[3] = {sd == 0 ? er[0] : -er[0], sd == 0 ? er[1] : -er[1], 0.0};
          testcoef_t C;
          mortar_coef(M, sd, &F[sd], &F[1 - sd], ns, &C);
          for (int i = 0; i < ndl; ++i) yl[sd][i] += JxW * test_dot(M, B[sd], i / nc, i % nc, &C);
        }
      }
    for (int sd = 0; sd < 2; ++sd)
      if (want[sd])
        for (int i = 0; i < ndl; ++i) y[dofs[sd][i]] += yl[sd][i];
  }
  free(B[0]);
  free(B[1]);
  free(yl[0]);
  free(yl[1]);
}

/* Alg. Alg-diagonal for the mortar part: for each interface cell side and each
 * local DoF i, the unit vector e_i on that side (other side zero) is evaluated
 * at the mortar points and integrated; entry i is kept. */
static void mortar_diag(const mesh_t *M, double *y) {
  if (M->P.merged) return;
  int n = M->n, d = M->d, nc = M->nc, ndl = M->nd * nc;
  int nqz = (d == 3) ? n : 1;
  pbasis_t *B = (pbasis_t *)malloc(sizeof(pbasis_t));
  for (long s = 0; s < M->nseg; ++s) {
    const seg_t *sg = &M->segs[s];
    const cell_t *c[2] = {iface_cell(M, 0, sg->ct_rotor, sg->cz), iface_cell(M, 1, sg->ct_stator, sg->cz)};
    double len = sg->hi - sg->lo;
    for (int sd = 0; sd < 2; ++sd) {
      long dofs[MAXND * 4];
      cell_dofs(M, c[sd], dofs);
      for (int qz = 0; qz < nqz; ++qz)
        for (int qt = 0; qt < n; ++qt) {
          double th = sg->lo + M->gx[qt] * len;
          double xiz = (d == 3) ? M->gx[qz] : 0.0;
          double JxW = M->gw[qt] * M->P.r_if * len * ((d == 3) ? M->gw[qz] * M->dz : 1.0);
          double xi[3];
          mortar_xi(M, c[sd], sd, th, xiz, xi);
          phys_basis(M, c[sd], xi, B);
          double er[3] = {cos(th), sin(th), 0.0};
          double ns[3] = {sd == 0 ? er[0] : -er[0], sd == 0 ? er[1] : -er[1], 0.0};
          field_t Fz;
          memset(&Fz, 0, sizeof(Fz));
          for (int i = 0; i < ndl; ++i) {
            int a = i / nc, comp = i % nc;
            field_t Fi;
            memset(&Fi, 0, sizeof(Fi));
            if (comp < d) {
              Fi.u[comp] = B->phi[a];
              for (int e = 0; e < d; ++e) Fi.gu[comp][e] = B->g[a][e];
            } else {
              Fi.p = B->phi[a];
            }
            testcoef_t C;
            mortar_coef(M, sd, &Fi, &Fz, ns, &C);
            y[dofs[i]] += JxW * test_dot(M, B, a, comp, &C);
          }
        }
    }
  }
  free(B);
}

/* ------------------------------------------------------------------------ */
/* Exported entry points                                                     */
/* ------------------------------------------------------------------------ */

int orc_ndofs(const orc_params *P, int64_t *n_total, int64_t *n_rotor, int64_t *n_cells, int64_t *n_segments) {
  mesh_t M;
  int rc = mesh_build(P, &M);
  if (rc) { mesh_free(&M); return rc; }
  *n_total = M.ndofs;
  *n_rotor = P->merged ? M.ndofs : M.noff[1] * M.nc;
  if (n_cells) *n_cells = M.ncells;
  if (n_segments) *n_segments = M.nseg;
  mesh_free(&M);
  return 0;
}

int orc_constrained(const orc_params *P, unsigned char *mask) {
  mesh_t M;
  int rc = mesh_build(P, &M);
  if (!rc) memcpy(mask, M.cons, (size_t)M.ndofs);
  mesh_free(&M);
  return rc;
}

/* node coordinates (x, y, z) in the current (rotated) configuration */
int orc_node_coords(const orc_params *P, double *xyz) {
  mesh_t M;
  int rc = mesh_build(P, &M);
  if (rc) { mesh_free(&M); return rc; }
  for (long ci = 0; ci < M.ncells; ++ci) {
    const cell_t *c = &M.cells[ci];
    for (int a = 0; a < M.nd; ++a) {
      int a0, a1, a2;
      local_idx(&M, a, &a0, &a1, &a2);
      long node = cell_node(&M, c, a0, a1, a2);
      double xi[3] = {M.gll[a0], M.gll[a1], M.gll[a2]}, x[3], J[3][3], X2[3][3][3];
      geom(&M, c, xi, x, J, X2);
      xyz[3 * node + 0] = x[0];
      xyz[3 * node + 1] = x[1];
      xyz[3 * node + 2] = x[2];
    }
  }
  mesh_free(&M);
  return 0;
}

/* per-cell data for the closed-form pins: h, V, penalty (interface cells) */
int orc_cell_info(const orc_params *P, double *h, double *V, double *tau_pen, double *tau_side2) {
  mesh_t M;
  int rc = mesh_build(P, &M);
  if (rc) { mesh_free(&M); return rc; }
  for (long ci = 0; ci < M.ncells; ++ci) {
    if (h) h[ci] = M.cells[ci].h;
    if (V) V[ci] = cell_measure(&M, &M.cells[ci]);
    if (tau_pen) tau_pen[ci] = M.cells[ci].tau_pen;
  }
  if (tau_side2) { tau_side2[0] = M.tau_side[0]; tau_side2[1] = M.tau_side[1]; }
  mesh_free(&M);
  return 0;
}

/* mortar segments: (cz, rotor face, stator face, lo, hi) and the JxW of every
 * mortar quadrature point, in segment order */
int orc_segments(const orc_params *P, int32_t *ids, double *lohi, double *jxw) {
  mesh_t M;
  int rc = mesh_build(P, &M);
  if (rc) { mesh_free(&M); return rc; }
  int n = M.n, nqz = (M.d == 3) ? n : 1;
  for (long s = 0; s < M.nseg; ++s) {
    const seg_t *sg = &M.segs[s];
    if (ids) { ids[3 * s] = sg->cz; ids[3 * s + 1] = sg->ct_rotor; ids[3 * s + 2] = sg->ct_stator; }
    if (lohi) { lohi[2 * s] = sg->lo; lohi[2 * s + 1] = sg->hi; }
    if (jxw)
      for (int qz = 0; qz < nqz; ++qz)
        for (int qt = 0; qt < n; ++qt)
          jxw[(s * nqz + qz) * n + qt] =
              M.gw[qt] * M.P.r_if * (sg->hi - sg->lo) * ((M.d == 3) ? M.gw[qz] * M.dz : 1.0);
  }
  mesh_free(&M);
  return 0;
}

/* 1D rules, for their own pins */
int orc_rules(int n, double *gll, double *gx, double *gw) {
  if (n < 2 || n > MAXN) return -1;
  lobatto01(n, gll);
  gauss01(n, gx, gw);
  return 0;
}

int orc_lagrange(int n, const double *nodes, double t, double *L, double *dL, double *d2L) {
  if (n < 1 || n > MAXN) return -1;
  lagrange(n, nodes, t, L, dL, d2L);
  return 0;
}

/* physical basis of one cell at a reference point, for the geometry pins */
int orc_phys_basis(const orc_params *P, int64_t cell, const double *xi, double *phi, double *grad, double *lap,
                   double *x) {
  mesh_t M;
  int rc = mesh_build(P, &M);
  if (rc) { mesh_free(&M); return rc; }
  if (cell < 0 || cell >= M.ncells) { mesh_free(&M); return -1; }
  pbasis_t *B = (pbasis_t *)malloc(sizeof(pbasis_t));
  double xx[3] = {xi[0], xi[1], xi[2]};
  phys_basis(&M, &M.cells[cell], xx, B);
  for (int a = 0; a < M.nd; ++a) {
    phi[a] = B->phi[a];
    for (int e = 0; e < 3; ++e) grad[3 * a + e] = B->g[a][e];
    lap[a] = B->lap[a];
  }
  for (int e = 0; e < 3; ++e) x[e] = B->x[e];
  free(B);
  mesh_free(&M);
  return 0;
}

/* y = J(state) x: constrained columns read as zero, constrained rows y = x */
int orc_apply_jacobian(const orc_params *P, const double *state, const double *hist, const double *force,
                       const double *x, double *y) {
  mesh_t M;
  int rc = mesh_build(P, &M);
  if (rc) { mesh_free(&M); return rc; }
  memset(y, 0, sizeof(double) * M.ndofs);
  inputs_t in = {state, hist, force, x, NULL};
  volume_loop(&M, &in, MODE_JAC, NULL, y);
  double *xm = (double *)malloc(sizeof(double) * M.ndofs);
  for (long i = 0; i < M.ndofs; ++i) xm[i] = M.cons[i] ? 0.0 : x[i];
  mortar_loop(&M, xm, NULL, y);
  free(xm);
  for (long i = 0; i < M.ndofs; ++i)
    if (M.cons[i]) y[i] = x[i];
  mesh_free(&M);
  return 0;
}

/* selected rows of J(state) x (cells and segments that touch them only) */
int orc_apply_jacobian_rows(const orc_params *P, const double *state, const double *hist, const double *force,
                            const double *x, int64_t nrows, const int64_t *rows, double *out) {
  mesh_t M;
  int rc = mesh_build(P, &M);
  if (rc) { mesh_free(&M); return rc; }
  unsigned char *node_mark = (unsigned char *)calloc((size_t)M.nnodes, 1);
  unsigned char *cmask = (unsigned char *)calloc((size_t)M.ncells, 1);
  for (int64_t i = 0; i < nrows; ++i) node_mark[rows[i] / M.nc] = 1;
  for (long ci = 0; ci < M.ncells; ++ci) {
    const cell_t *c = &M.cells[ci];
    for (int a = 0; a < M.nd && !cmask[ci]; ++a) {
      int a0, a1, a2;
      local_idx(&M, a, &a0, &a1, &a2);
      if (node_mark[cell_node(&M, c, a0, a1, a2)]) cmask[ci] = 1;
    }
  }
  double *y = (double *)calloc((size_t)M.ndofs, sizeof(double));
  inputs_t in = {state, hist, force, x, NULL};
  volume_loop(&M, &in, MODE_JAC, cmask, y);
  double *xm = (double *)malloc(sizeof(double) * M.ndofs);
  for (long i = 0; i < M.ndofs; ++i) xm[i] = M.cons[i] ? 0.0 : x[i];
  mortar_loop(&M, xm, cmask, y);
  for (int64_t i = 0; i < nrows; ++i) out[i] = M.cons[rows[i]] ? x[rows[i]] : y[rows[i]];
  free(xm);
  free(y);
  free(cmask);
  free(node_mark);
  mesh_free(&M);
  return 0;
}

/* nonlinear residual; tau from tau_state when given (frozen), else from state;
 * constrained rows are zero */
int orc_residual(const orc_params *P, const double *state, const double *hist, const double *force,
                 const double *tau_state, double *res) {
  mesh_t M;
  int rc = mesh_build(P, &M);
  if (rc) { mesh_free(&M); return rc; }
  memset(res, 0, sizeof(double) * M.ndofs);
  inputs_t in = {state, hist, force, NULL, tau_state};
  volume_loop(&M, &in, MODE_RES, NULL, res);
  mortar_loop(&M, state, NULL, res);
  for (long i = 0; i < M.ndofs; ++i)
    if (M.cons[i]) res[i] = 0.0;
  mesh_free(&M);
  return 0;
}

/* diagonal of J(state): volume columns plus Alg. Alg-diagonal; constrained = 1 */
int orc_diagonal(const orc_params *P, const double *state, const double *hist, const double *force, double *diag) {
  mesh_t M;
  int rc = mesh_build(P, &M);
  if (rc) { mesh_free(&M); return rc; }
  memset(diag, 0, sizeof(double) * M.ndofs);
  inputs_t in = {state, hist, force, NULL, NULL};
  volume_loop(&M, &in, MODE_DIAG, NULL, diag);
  mortar_diag(&M, diag);
  for (long i = 0; i < M.ndofs; ++i)
    if (M.cons[i]) diag[i] = 1.0;
  mesh_free(&M);
  return 0;
}

/* Assembled J(state) as COO triplets (duplicates to be summed by the caller).
 * Volume: element matrices column by column.  Mortar: Alg. Alg-matrix, each
 * trial DoF of either side is evaluated at the mortar points and integrated
 * against the test functions of both sides.  Constrained rows become identity
 * rows, constrained columns are dropped.  Call with rows == NULL to get the
 * capacity needed. */
int orc_assemble(const orc_params *P, const double *state, const double *hist, const double *force, int64_t cap,
                 int64_t *rows, int64_t *cols, double *vals, int64_t *count) {
  mesh_t M;
  int rc = mesh_build(P, &M);
  if (rc) { mesh_free(&M); return rc; }
  int d = M.d, nc = M.nc, ndl = M.nd * nc, n = M.n;
  int64_t need = (int64_t)M.ncells * ndl * ndl + (int64_t)M.nseg * 4 * ndl * ndl + M.ndofs;
  if (!rows) { *count = need; mesh_free(&M); return 0; }
  if (cap < need) { mesh_free(&M); return -4; }
  int64_t cnt = 0;
  pbasis_t *B = (pbasis_t *)malloc(sizeof(pbasis_t));
  double *K = (double *)malloc(sizeof(double) * ndl * ndl);
  for (long ci = 0; ci < M.ncells; ++ci) {
    const cell_t *c = &M.cells[ci];
    long dofs[MAXND * 4];
    double Sl[MAXND * 4], Hl[MAXND * 4], Fl[MAXND * 4];
    cell_dofs(&M, c, dofs);
    gather(&M, dofs, state, 0, Sl);
    gather(&M, dofs, hist, 0, Hl);
    gather(&M, dofs, force, 0, Fl);
    memset(K, 0, sizeof(double) * ndl * ndl);
    for (int q = 0; q < M.nd; ++q) {
      double xi[3];
      double wq = cell_qp(&M, q, xi);
      phys_basis(&M, c, xi, B);
      double JxW = wq * fabs(B->detJ);
      field_t S;
      eval_field(&M, B, Sl, &S);
      double w[3], hh[3], f[3];
      ale_velocity(&M, c, B->x, w);
      interp_vec(&M, B, (hist && !M.P.steady) ? Hl : NULL, hh);
      if (M.P.mms) mms_forcing(&M, B->x, w, f);
      else interp_vec(&M, B, force ? Fl : NULL, f);
      double a[3] = {0, 0, 0};
      for (int m = 0; m < d; ++m) a[m] = S.u[m] - w[m];
      double tau = tau_u(&M, a, c->h);
      for (int j = 0; j < ndl; ++j) {
        int b = j / nc, cb = j % nc;
        field_t T;
        memset(&T, 0, sizeof(T));
        if (cb < d) {
          T.u[cb] = B->phi[b];
          for (int e = 0; e < d; ++e) T.gu[cb][e] = B->g[b][e];
          T.lu[cb] = B->lap[b];
        } else {
          T.p = B->phi[b];
          for (int e = 0; e < d; ++e) T.gp[e] = B->g[b][e];
        }
        testcoef_t C;
        pw_jacobian(&M, &S, hh, f, w, tau, &T, &C);
        for (int i = 0; i < ndl; ++i) K[i * ndl + j] += JxW * test_dot(&M, B, i / nc, i % nc, &C);
      }
    }
    for (int i = 0; i < ndl; ++i)
      for (int j = 0; j < ndl; ++j) {
        if (M.cons[dofs[i]] || M.cons[dofs[j]]) continue;
        rows[cnt] = dofs[i];
        cols[cnt] = dofs[j];
        vals[cnt] = K[i * ndl + j];
        ++cnt;
      }
  }
  if (!M.P.merged) {
    int nqz = (d == 3) ? n : 1;
    pbasis_t *Bs[2];
    Bs[0] = (pbasis_t *)malloc(sizeof(pbasis_t));
    Bs[1] = (pbasis_t *)malloc(sizeof(pbasis_t));
    double *Km = (double *)malloc(sizeof(double) * ndl * ndl);
    for (long s = 0; s < M.nseg; ++s) {
      const seg_t *sg = &M.segs[s];
      const cell_t *c[2] = {iface_cell(&M, 0, sg->ct_rotor, sg->cz), iface_cell(&M, 1, sg->ct_stator, sg->cz)};
      long dofs[2][MAXND * 4];
      cell_dofs(&M, c[0], dofs[0]);
      cell_dofs(&M, c[1], dofs[1]);
      double len = sg->hi - sg->lo;
      for (int ts = 0; ts < 2; ++ts)     /* test side */
        for (int tr = 0; tr < 2; ++tr) { /* trial side */
          memset(Km, 0, sizeof(double) * ndl * ndl);
          for (int qz = 0; qz < nqz; ++qz)
            for (int qt = 0; qt < n; ++qt) {
              double th = sg->lo + M.gx[qt] * len;
              double xiz = (d == 3) ? M.gx[qz] : 0.0;
              double JxW = M.gw[qt] * M.P.r_if * len * ((d == 3) ? M.gw[qz] * M.dz : 1.0);
              for (int sd = 0; sd < 2; ++sd) {
                double xi[3];
                mortar_xi(&M, c[sd], sd, th, xiz, xi);
                phys_basis(&M, c[sd], xi, Bs[sd]);
              }
              double er[3] = {cos(th), sin(th), 0.0};
              double ns[3] = {ts == 0 ? er[0] : -er[0], ts == 0 ? er[1] : -er[1], 0.0};
              for (int j = 0; j < ndl; ++j) {
                int b = j / nc, cb = j % nc;
                field_t F[2];
                memset(F, 0, sizeof(F));
                field_t *Ft = &F[tr];
                if (cb < d) {
                  Ft->u[cb] = Bs[tr]->phi[b];
                  for (int e = 0; e < d; ++e) Ft->gu[cb][e] = Bs[tr]->g[b][e];
                } else {
                  Ft->p = Bs[tr]->phi[b];
                }
                testcoef_t C;
                mortar_coef(&M, ts, &F[ts], &F[1 - ts], ns, &C);
                for (int i = 0; i < ndl; ++i) Km[i * ndl + j] += JxW * test_dot(&M, Bs[ts], i / nc, i % nc, &C);
              }
            }
          for (int i = 0; i < ndl; ++i)
            for (int j = 0; j < ndl; ++j) {
              if (M.cons[dofs[ts][i]] || M.cons[dofs[tr][j]]) continue;
              rows[cnt] = dofs[ts][i];
              cols[cnt] = dofs[tr][j];
              vals[cnt] = Km[i * ndl + j];
              ++cnt;
            }
        }
    }
    free(Km);
    free(Bs[0]);
    free(Bs[1]);
  }
  for (long i = 0; i < M.ndofs; ++i)
    if (M.cons[i]) {
      rows[cnt] = i;
      cols[cnt] = i;
      vals[cnt] = 1.0;
      ++cnt;
    }
  *count = cnt;
  free(K);
  free(B);
  mesh_free(&M);
  return 0;
}

/* nodal interpolant of the 2D manufactured solution (Sec. 4.1) */
int orc_mms_interpolate(const orc_params *P, double *vec) {
  mesh_t M;
  int rc = mesh_build(P, &M);
  if (rc) { mesh_free(&M); return rc; }
  if (M.d != 2) { mesh_free(&M); return -1; }
  for (long ci = 0; ci < M.ncells; ++ci) {
    const cell_t *c = &M.cells[ci];
    for (int a = 0; a < M.nd; ++a) {
      int a0, a1, a2;
      local_idx(&M, a, &a0, &a1, &a2);
      long node = cell_node(&M, c, a0, a1, a2);
      double xi[3] = {M.gll[a0], M.gll[a1], 0.0}, x[3], J[3][3], X2[3][3][3];
      geom(&M, c, xi, x, J, X2);
      double u[3], gu[3][3], lu[3], p, gp[3];
      mms_fields(x, u, gu, lu, &p, gp);
      vec[node * M.nc + 0] = u[0];
      vec[node * M.nc + 1] = u[1];
      vec[node * M.nc + 2] = p;
    }
  }
  mesh_free(&M);
  return 0;
}

/* L2 errors of velocity and of mean-free pressure against the manufactured
 * solution, with an (n+3)-point Gauss rule per direction */
int orc_mms_errors(const orc_params *P, const double *sol, double *err) {
  mesh_t M;
  int rc = mesh_build(P, &M);
  if (rc) { mesh_free(&M); return rc; }
  if (M.d != 2) { mesh_free(&M); return -1; }
  int nq = M.n + 3;
  double qx[MAXN + 4], qw[MAXN + 4];
  if (nq > MAXN) nq = MAXN;
  gauss01(nq, qx, qw);
  pbasis_t *B = (pbasis_t *)malloc(sizeof(pbasis_t));
  double eu = 0.0, area = 0.0, pmean = 0.0, ep = 0.0;
  for (int pass = 0; pass < 2; ++pass)
    for (long ci = 0; ci < M.ncells; ++ci) {
      const cell_t *c = &M.cells[ci];
      long dofs[MAXND * 4];
      double Sl[MAXND * 4];
      cell_dofs(&M, c, dofs);
      gather(&M, dofs, sol, 0, Sl);
      for (int q1 = 0; q1 < nq; ++q1)
        for (int q0 = 0; q0 < nq; ++q0) {
          double xi[3] = {qx[q0], qx[q1], 0.0};
          phys_basis(&M, c, xi, B);
          double JxW = qw[q0] * qw[q1] * fabs(B->detJ);
          field_t S;
          eval_field(&M, B, Sl, &S);
          double u[3], gu[3][3], lu[3], p, gp[3];
          mms_fields(B->x, u, gu, lu, &p, gp);
          if (pass == 0) {
            eu += JxW * ((S.u[0] - u[0]) * (S.u[0] - u[0]) + (S.u[1] - u[1]) * (S.u[1] - u[1]));
            pmean += JxW * (S.p - p);
            area += JxW;
          } else {
            double e = S.p - p - pmean / area;
            ep += JxW * e * e;
          }
        }
    }
  err[0] = sqrt(eu);
  err[1] = sqrt(ep);
  free(B);
  mesh_free(&M);
  return 0;
}
