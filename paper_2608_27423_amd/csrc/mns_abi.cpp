// extern "C" entry points of libmortarns (declared in include/mortarns.h).
// Every entry point validates its arguments, maps failures to MNS_ERR_* codes
// and never lets a C++ exception cross the interface.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <new>
#include <string>

#include "mns_internal.hpp"

using namespace mns;

int mns_build_handle(const mns_mesh_desc* d, hipStream_t stream, mns_handle* h);
int mns_rotate_tables(mns_handle* h, double theta, double omega, hipStream_t s);
int mns_solve_impl(mns_handle* h, const double* rhs, double* x, const mns_solve_opts* o, mns_solve_report* rep,
                   hipStream_t s);

static void free_events(mns_handle* h) {
  for (int c = 0; c < 3; ++c) {
    for (hipEvent_t e : h->ev[c]) (void)hipEventDestroy(e);
    h->ev[c].clear();
    h->ev_used[c] = 0;
  }
  h->timing_cap = 0;
}

static void free_all(mns_handle* h) {
  free_events(h);
  if (h->ev_fork) (void)hipEventDestroy(h->ev_fork);
  if (h->ev_join) (void)hipEventDestroy(h->ev_join);
  if (h->aux) (void)hipStreamDestroy(h->aux);
  if (h->cap) (void)hipStreamDestroy(h->cap);
  h->ev_fork = h->ev_join = nullptr;
  h->aux = h->cap = nullptr;
  mns::mg_free(h);
  void** ptrs[] = {(void**)&h->d_hcell64, (void**)&h->d_hcell32, (void**)&h->d_trig64, (void**)&h->d_trig32,
                   &h->d_mtab64, &h->d_mtab32, (void**)&h->d_mtrig64, (void**)&h->d_mtrig32, (void**)&h->d_cons,
                   (void**)&h->d_lin64, (void**)&h->d_lin32, (void**)&h->d_hist_buf, (void**)&h->d_force_buf,
                   (void**)&h->ws64, (void**)&h->ws32, (void**)&h->d_E64, (void**)&h->d_E32, (void**)&h->d_Em64,
                   (void**)&h->d_Em32, (void**)&h->d_diag64, (void**)&h->d_diag32, (void**)&h->d_red, (void**)&h->d_gm,
                   (void**)&h->d_step, (void**)&h->d_state, (void**)&h->d_linc64, (void**)&h->d_linc32,
                   (void**)&h->d_state32, (void**)&h->d_xnode, (void**)&h->d_geo64, (void**)&h->d_geo32,
                   (void**)&h->d_geox, (void**)&h->d_hiso, (void**)&h->d_iso_flag, (void**)&h->d_mgeo64,
                   (void**)&h->d_mgeo32};
  for (void** p : ptrs) {
    if (*p) (void)hipFree(*p);
    *p = nullptr;
  }
  h->d_hist = h->d_force = nullptr;
  if (h->h_red) (void)hipHostFree(h->h_red);
  h->h_red = nullptr;
}

static bool aligned(const void* p, size_t a) { return p && ((uintptr_t)p % a) == 0; }

static hipStream_t as_stream(void* s) { return (hipStream_t)s; }

// every instance must hold a linearization at its current angle: a rotation
// of a member handle after mns_batch_create clears it until it is relinearized
static int batch_check_linearized(mns_batch* b) {
  for (size_t i = 0; i < b->hs.size(); ++i)
    if (!b->hs[i]->rotated || !b->hs[i]->linearized) {
      b->err = "batch: instance " + std::to_string(i) +
               " has no linearization at its current angle (call mns_set_linearization after mns_rotate_rotor)";
      return MNS_ERR_NOT_LINEARIZED;
    }
  return MNS_OK;
}

extern "C" {

int mns_setup_mesh(const mns_mesh_desc* desc, void* stream, mns_handle** out) {
  if (!desc || !out) return MNS_ERR_INVALID_ARG;
  *out = nullptr;
  mns_handle* h = new (std::nothrow) mns_handle();
  if (!h) return MNS_ERR_HIP;
  int rc;
  try {
    rc = mns_build_handle(desc, as_stream(stream), h);
  } catch (...) {
    rc = MNS_ERR_HIP;
  }
  if (rc != MNS_OK) {
    // keep the handle so the caller can read the message; it holds no device memory
    free_all(h);
    *out = h;
    return rc;
  }
  // device address of the allocation-free apply's scratch array on this
  // device (looked up once per device; a failure here is reported by that
  // entry point, which tries again)
  void* scratch = nullptr;
  (void)mns::scratch_pointer(&scratch, nullptr);
  *out = h;
  return MNS_OK;
}

int mns_n_dofs(const mns_handle* h, int64_t* n_total, int64_t* n_rotor) {
  if (!h || !n_total || !n_rotor) return MNS_ERR_INVALID_ARG;
  *n_total = h->ndofs;
  *n_rotor = h->node_off1 * h->nc;
  return MNS_OK;
}

int mns_rotate_rotor(mns_handle* h, double theta, double omega, void* stream) {
  if (!h) return MNS_ERR_INVALID_ARG;
  if (h->ndofs == 0 || !h->d_mtab64) return set_error(h, MNS_ERR_INVALID_ARG, "handle was not set up");
  if (!std::isfinite(theta) || !std::isfinite(omega))
    return set_error(h, MNS_ERR_INVALID_ARG, "theta and omega must be finite");
  int rc;
  try {
    rc = mns_rotate_tables(h, theta, omega, as_stream(stream));
    if (rc == MNS_OK) rc = mns::iso_rotate(h, theta, as_stream(stream));
  } catch (...) {
    rc = set_error(h, MNS_ERR_HIP, "exception in rotate");
  }
  h->rotated = rc == MNS_OK;
  ++h->lin_version;
  h->linearized = false;
  h->diag_valid = false;
  return rc;
}

int mns_set_node_positions(mns_handle* h, const double* xyz, int64_t n_nodes, void* stream) {
  if (!h) return MNS_ERR_INVALID_ARG;
  if (h->ndofs == 0 || !h->d_mtab64) return set_error(h, MNS_ERR_INVALID_ARG, "handle was not set up");
  int rc;
  try {
    // a multigrid hierarchy holds coarse levels of the old geometry
    mns::mg_free(h);
    rc = mns::iso_set_nodes(h, xyz, n_nodes, as_stream(stream));
  } catch (...) {
    rc = set_error(h, MNS_ERR_HIP, "exception in set_node_positions");
  }
  // the geometry changed: the next apply needs a rotation and a linearization
  h->rotated = false;
  ++h->lin_version;
  h->linearized = false;
  h->diag_valid = false;
  return rc;
}

int mns_set_linearization_kind(mns_handle* h, int kind) {
  if (!h) return MNS_ERR_INVALID_ARG;
  if (kind != MNS_LIN_NEWTON && kind != MNS_LIN_PICARD)
    return set_error(h, MNS_ERR_INVALID_ARG, "kind must be MNS_LIN_NEWTON or MNS_LIN_PICARD");
  h->picard = kind == MNS_LIN_PICARD;
  return MNS_OK;
}

int mns_set_linearization(mns_handle* h, const double* state, const double* u_hist, const double* force,
                          void* stream) {
  if (!h) return MNS_ERR_INVALID_ARG;
  if (!h->rotated) return set_error(h, MNS_ERR_NO_ROTATION, "call mns_rotate_rotor first");
  if (!aligned(state, 8)) return set_error(h, MNS_ERR_INVALID_ARG, "state must be a non-null 8-byte aligned pointer");
  if ((u_hist && !aligned(u_hist, 8)) || (force && !aligned(force, 8)))
    return set_error(h, MNS_ERR_INVALID_ARG, "history/force must be 8-byte aligned");
  hipStream_t s = as_stream(stream);
  const int LS = h->dim == 3 ? LinLayout<3>::SIZE : LinLayout<2>::SIZE;
  const size_t nlin = (size_t)h->ncells * (size_t)(h->dim == 3 ? h->n * h->n * h->n : h->n * h->n) * LS;
  hipError_t e;
  // keep copies of the history and force for mns_apply_residual; their
  // buffers are allocated by the first call that passes them and kept
  const double* srcs[2] = {u_hist, force};
  double** bufs[2] = {&h->d_hist_buf, &h->d_force_buf};
  double** dsts[2] = {&h->d_hist, &h->d_force};
  for (int i = 0; i < 2; ++i) {
    if (srcs[i]) {
      if (!*bufs[i] && (e = hipMalloc((void**)bufs[i], h->ndofs * sizeof(double))) != hipSuccess)
        return set_error(h, MNS_ERR_HIP, std::string("hipMalloc: ") + hipGetErrorString(e));
      if ((e = hipMemcpyAsync(*bufs[i], srcs[i], h->ndofs * sizeof(double), hipMemcpyDeviceToDevice, s)) !=
          hipSuccess)
        return set_error(h, MNS_ERR_HIP, std::string("copy: ") + hipGetErrorString(e));
      *dsts[i] = *bufs[i];
    } else {
      *dsts[i] = nullptr;
    }
  }
  // the state is kept for the multigrid hierarchy (injected to coarse levels)
  if ((e = hipMemcpyAsync(h->d_state, state, h->ndofs * sizeof(double), hipMemcpyDeviceToDevice, s)) != hipSuccess)
    return set_error(h, MNS_ERR_HIP, std::string("copy state: ") + hipGetErrorString(e));
  ++h->lin_version;
  int rc = launch_linearize<double>(h, state, h->desc.steady ? nullptr : h->d_hist, h->d_force, h->d_lin64, s);
  if (rc) return rc;
  rc = mns::launch_cast_f64_f32(h->d_lin64, h->d_lin32, (int64_t)nlin, s);
  if (rc) return set_error(h, rc, "cast");
  // linearization source C: tau and tau R per point, the state in FP32
  if (h->d_linc64) {
    if ((rc = mns::launch_lin_compact(h, s))) return rc;
    if ((rc = mns::launch_cast_f64_f32(state, h->d_state32, h->ndofs, s))) return set_error(h, rc, "cast");
  }
  h->lin_picard = h->picard;
  h->linearized = true;
  h->diag_valid = false;
  return MNS_OK;
}

int mns_batch_create(mns_handle* const* handles, int count, mns_batch** batch) {
  if (!batch) return MNS_ERR_INVALID_ARG;
  *batch = nullptr;
  if (!handles || count < 1 || count > 65536) return MNS_ERR_INVALID_ARG;
  for (int i = 0; i < count; ++i) {
    mns_handle* h = handles[i];
    if (!h) return MNS_ERR_INVALID_ARG;
    if (!h->rotated || !h->linearized)
      return set_error(h, MNS_ERR_NOT_LINEARIZED, "batch: rotate and linearize every handle first");
    if (!h->equal_rings)
      return set_error(h, MNS_ERR_UNSUPPORTED, "batch: instances need equal interface cell counts");
  }
  auto* b = new mns_batch();
  b->hs.assign(handles, handles + count);
  // one group per (dimension, degree, geometry kind), in the order of first
  // appearance
  for (int i = 0; i < count; ++i) {
    mns_batch_group* g = nullptr;
    for (auto& x : b->groups)
      if (x.dim == handles[i]->dim && x.k == handles[i]->k && x.iso == handles[i]->iso) g = &x;
    if (!g) {
      b->groups.emplace_back();
      g = &b->groups.back();
      g->dim = handles[i]->dim;
      g->k = handles[i]->k;
      g->iso = handles[i]->iso;
    }
    g->members.push_back(i);
  }
  for (int i = 0; i < count; ++i) {
    b->offsets.push_back(b->ndofs);
    b->ndofs += handles[i]->ndofs;
  }
  int rc;
  try {
    rc = mns::batch_build(b);
  } catch (...) {
    rc = MNS_ERR_HIP;
    b->err = "exception in batch setup";
  }
  if (rc) {
    (void)set_error(handles[0], rc, b->err);
    mns_batch_destroy(b);
    return rc;
  }
  *batch = b;
  return MNS_OK;
}

int mns_batch_n_dofs(const mns_batch* b, int64_t* n_total) {
  if (!b || !n_total) return MNS_ERR_INVALID_ARG;
  *n_total = b->ndofs;
  return MNS_OK;
}

int mns_batch_apply_jacobian(mns_batch* b, int precision, const void* src, void* dst, void* stream) {
  if (!b) return MNS_ERR_INVALID_ARG;
  if (int rc = batch_check_linearized(b)) return rc;
  if (src == dst) {
    b->err = "src and dst must not overlap";
    return MNS_ERR_INVALID_ARG;
  }
  try {
    if (precision == MNS_F64) {
      if (!aligned(src, 8) || !aligned(dst, 8)) {
        b->err = "misaligned or null vector";
        return MNS_ERR_INVALID_ARG;
      }
      return mns::launch_batch_jacobian<double>(b, (const double*)src, (double*)dst, as_stream(stream));
    }
    if (precision == MNS_F32) {
      if (!aligned(src, 4) || !aligned(dst, 4)) {
        b->err = "misaligned or null vector";
        return MNS_ERR_INVALID_ARG;
      }
      return mns::launch_batch_jacobian<float>(b, (const float*)src, (float*)dst, as_stream(stream));
    }
  } catch (...) {
    b->err = "exception in batch apply";
    return MNS_ERR_HIP;
  }
  b->err = "precision must be MNS_F64 or MNS_F32";
  return MNS_ERR_INVALID_ARG;
}

const char* mns_batch_last_error(const mns_batch* b) { return b ? b->err.c_str() : "null batch"; }

int mns_batch_solve(mns_batch* b, const double* rhs, double* x, const mns_solve_opts* opts,
                    mns_solve_report* reports, void* stream) {
  if (!b) return MNS_ERR_INVALID_ARG;
  if (int rc = batch_check_linearized(b)) return rc;
  if (!aligned(rhs, 8) || !aligned(x, 8) || rhs == x) {
    b->err = "rhs/x must be distinct 8-byte aligned pointers";
    return MNS_ERR_INVALID_ARG;
  }
  mns_solve_opts o;
  mns_default_solve_opts(&o);
  if (opts) o = *opts;
  if (!(o.rtol > 0) || o.restart < 1 || o.restart > 200 || o.maxit < 1 || o.cheb_degree < 1 || o.cheb_degree > 32 ||
      !(o.cheb_range > 1) || o.eig_iters < 1 ||
      (o.precond != -1 && o.precond != MNS_F64 && o.precond != MNS_F32 && o.precond != MNS_PRECOND_MG &&
       o.precond != MNS_PRECOND_MG64) ||
      !(o.cheb_lambda_factor >= 1.0 && o.cheb_lambda_factor <= 4.0) || o.mg_levels < 0 || o.mg_levels > 16 ||
      o.mg_coarse_degree < 1 || o.mg_coarse_degree > 1000 || o.mg_smooth_degree < 1 || o.mg_smooth_degree > 32 ||
      !(o.mg_smooth_range > 1) ||
      (o.mg_coarse_linearization != MNS_LIN_NEWTON && o.mg_coarse_linearization != MNS_LIN_PICARD) ||
      (o.mg_fine_linearization != MNS_LIN_NEWTON && o.mg_fine_linearization != MNS_LIN_PICARD) ||
      (o.use_graph != 0 && o.use_graph != 1) || (o.mg_coarse_direct != 0 && o.mg_coarse_direct != 1)) {
    b->err = "invalid batch solve options (restart 1..200, Chebyshev and smoother degrees 1..32)";
    return MNS_ERR_INVALID_ARG;
  }
  try {
    return mns::batch_solve_impl(b, rhs, x, &o, reports, as_stream(stream));
  } catch (...) {
    b->err = "exception in batch solve";
    return MNS_ERR_HIP;
  }
}

void mns_batch_destroy(mns_batch* b) {
  if (!b) return;
  mns::batch_solver_free(b);
  for (auto& g : b->groups) {
    if (g.d_items64) (void)hipFree(g.d_items64);
    if (g.d_items32) (void)hipFree(g.d_items32);
    if (g.d_prefix) (void)hipFree(g.d_prefix);
  }
  delete b;
}

int mns_apply_jacobian(mns_handle* h, int precision, const void* src, void* dst, void* stream) {
  if (!h) return MNS_ERR_INVALID_ARG;
  if (!h->linearized) return set_error(h, MNS_ERR_NOT_LINEARIZED, "call mns_set_linearization first");
  if (src == dst) return set_error(h, MNS_ERR_INVALID_ARG, "src and dst must not overlap");
  try {
    if (precision == MNS_F64) {
      if (!aligned(src, 8) || !aligned(dst, 8)) return set_error(h, MNS_ERR_INVALID_ARG, "misaligned or null vector");
      return launch_jacobian<double>(h, (const double*)src, (double*)dst, as_stream(stream));
    }
    if (precision == MNS_F32) {
      if (!aligned(src, 4) || !aligned(dst, 4)) return set_error(h, MNS_ERR_INVALID_ARG, "misaligned or null vector");
      return launch_jacobian<float>(h, (const float*)src, (float*)dst, as_stream(stream));
    }
  } catch (...) {
    return set_error(h, MNS_ERR_HIP, "exception in apply_jacobian");
  }
  return set_error(h, MNS_ERR_INVALID_ARG, "precision must be MNS_F64 or MNS_F32");
}

int mns_apply_jacobian_noalloc(mns_handle* h, int precision, const void* src, void* dst, void* stream) {
  if (!h) return MNS_ERR_INVALID_ARG;
  if (!h->linearized) return set_error(h, MNS_ERR_NOT_LINEARIZED, "call mns_set_linearization first");
  if (src == dst) return set_error(h, MNS_ERR_INVALID_ARG, "src and dst must not overlap");
  try {
    if (precision == MNS_F64) {
      if (!aligned(src, 8) || !aligned(dst, 8)) return set_error(h, MNS_ERR_INVALID_ARG, "misaligned or null vector");
      return launch_jacobian_noalloc<double>(h, (const double*)src, (double*)dst, as_stream(stream));
    }
    if (precision == MNS_F32) {
      if (!aligned(src, 4) || !aligned(dst, 4)) return set_error(h, MNS_ERR_INVALID_ARG, "misaligned or null vector");
      return launch_jacobian_noalloc<float>(h, (const float*)src, (float*)dst, as_stream(stream));
    }
  } catch (...) {
    return set_error(h, MNS_ERR_HIP, "exception in apply_jacobian_noalloc");
  }
  return set_error(h, MNS_ERR_INVALID_ARG, "precision must be MNS_F64 or MNS_F32");
}

int mns_assemble_matrix(mns_handle* h, double* A, int64_t lda, void* stream) {
  if (!h) return MNS_ERR_INVALID_ARG;
  if (!h->linearized) return set_error(h, MNS_ERR_NOT_LINEARIZED, "call mns_set_linearization first");
  if (!aligned(A, 8) || lda < h->ndofs) return set_error(h, MNS_ERR_INVALID_ARG, "A must be aligned with lda >= n");
  if (h->ndofs > 32768) return set_error(h, MNS_ERR_UNSUPPORTED, "dense assembly is limited to 32,768 DoFs");
  try {
    return mns::assemble_matrix(h, A, (long long)lda, as_stream(stream));
  } catch (...) {
    return set_error(h, MNS_ERR_HIP, "exception in assemble_matrix");
  }
}

int mns_apply_residual(mns_handle* h, const double* state, double* res, void* stream) {
  if (!h) return MNS_ERR_INVALID_ARG;
  if (!h->rotated) return set_error(h, MNS_ERR_NO_ROTATION, "call mns_rotate_rotor first");
  if (!aligned(state, 8) || !aligned(res, 8) || state == res)
    return set_error(h, MNS_ERR_INVALID_ARG, "state/res must be distinct 8-byte aligned pointers");
  try {
    return launch_residual(h, state, res, as_stream(stream));
  } catch (...) {
    return set_error(h, MNS_ERR_HIP, "exception in apply_residual");
  }
}

int mns_compute_diagonal(mns_handle* h, int precision, void* diag, void* stream) {
  if (!h) return MNS_ERR_INVALID_ARG;
  if (!h->linearized) return set_error(h, MNS_ERR_NOT_LINEARIZED, "call mns_set_linearization first");
  try {
    if (precision == MNS_F64) {
      if (!aligned(diag, 8)) return set_error(h, MNS_ERR_INVALID_ARG, "misaligned or null vector");
      return launch_diagonal<double>(h, (double*)diag, as_stream(stream));
    }
    if (precision == MNS_F32) {
      if (!aligned(diag, 4)) return set_error(h, MNS_ERR_INVALID_ARG, "misaligned or null vector");
      return launch_diagonal<float>(h, (float*)diag, as_stream(stream));
    }
  } catch (...) {
    return set_error(h, MNS_ERR_HIP, "exception in compute_diagonal");
  }
  return set_error(h, MNS_ERR_INVALID_ARG, "precision must be MNS_F64 or MNS_F32");
}

void mns_default_solve_opts(mns_solve_opts* o) {
  if (!o) return;
  o->rtol = 1e-8;
  o->restart = 50;
  o->maxit = 2000;
  o->precond = MNS_F32;
  o->cheb_degree = 4;
  o->cheb_range = 30.0;
  o->eig_iters = 20;
  o->mg_levels = 0;
  o->mg_smooth_degree = 2;
  o->mg_smooth_range = 5.0;
  o->mg_coarse_degree = 16;
  o->mg_coarse_linearization = MNS_LIN_NEWTON;
  o->mg_fine_linearization = MNS_LIN_NEWTON;
  o->use_graph = 1;
  o->cheb_lambda_factor = 1.05;
  o->mg_coarse_direct = 1;
}

int mns_solve(mns_handle* h, const double* rhs, double* x, const mns_solve_opts* opts, mns_solve_report* report,
              void* stream) {
  if (!h) return MNS_ERR_INVALID_ARG;
  if (!h->linearized) return set_error(h, MNS_ERR_NOT_LINEARIZED, "call mns_set_linearization first");
  if (!aligned(rhs, 8) || !aligned(x, 8) || rhs == x)
    return set_error(h, MNS_ERR_INVALID_ARG, "rhs/x must be distinct 8-byte aligned pointers");
  mns_solve_opts o;
  mns_default_solve_opts(&o);
  if (opts) o = *opts;
  if (!(o.rtol > 0) || o.restart < 1 || o.restart > 1000 || o.maxit < 1 || o.cheb_degree < 1 ||
      o.cheb_degree > 100 || !(o.cheb_range > 1) || o.eig_iters < 1 ||
      (o.precond != -1 && o.precond != MNS_F64 && o.precond != MNS_F32 && o.precond != MNS_PRECOND_MG &&
       o.precond != MNS_PRECOND_MG64) ||
      o.mg_levels < 0 || o.mg_levels > 16 || o.mg_coarse_degree < 1 || o.mg_coarse_degree > 1000 ||
      o.mg_smooth_degree < 1 || o.mg_smooth_degree > 100 || !(o.mg_smooth_range > 1) ||
      (o.mg_coarse_linearization != MNS_LIN_NEWTON && o.mg_coarse_linearization != MNS_LIN_PICARD) ||
      (o.mg_fine_linearization != MNS_LIN_NEWTON && o.mg_fine_linearization != MNS_LIN_PICARD) ||
      (o.use_graph != 0 && o.use_graph != 1) || !(o.cheb_lambda_factor >= 1.0 && o.cheb_lambda_factor <= 4.0) ||
      (o.mg_coarse_direct != 0 && o.mg_coarse_direct != 1))
    return set_error(h, MNS_ERR_INVALID_ARG, "invalid solve options");
  mns_solve_report rep{};
  int rc;
  try {
    rc = mns_solve_impl(h, rhs, x, &o, &rep, as_stream(stream));
  } catch (...) {
    rc = set_error(h, MNS_ERR_HIP, "exception in solve");
  }
  if (report) *report = rep;
  return rc;
}

void mns_default_step_opts(mns_step_opts* o) {
  if (!o) return;
  o->newton_rtol = 1e-8;
  o->newton_atol = 1e-13;
  o->max_newton = 8;
  mns_default_solve_opts(&o->linear);
  o->linear.rtol = 1e-6;
}

int mns_bdf2_step(mns_handle* h, double theta_next, double omega, const double* u_n, const double* u_nm1,
                  const double* force, double* u_next, const mns_step_opts* opts, mns_step_report* report,
                  void* stream) {
  if (!h) return MNS_ERR_INVALID_ARG;
  if (h->ndofs == 0) return set_error(h, MNS_ERR_INVALID_ARG, "handle was not set up");
  if (h->desc.steady) return set_error(h, MNS_ERR_INVALID_ARG, "the mesh description is steady (no time step)");
  if (!aligned(u_n, 8) || !aligned(u_next, 8) || (u_nm1 && !aligned(u_nm1, 8)) || (force && !aligned(force, 8)) ||
      u_next == u_n || u_next == u_nm1 || u_next == force)
    return set_error(h, MNS_ERR_INVALID_ARG, "vectors must be 8-byte aligned and u_next distinct from the inputs");
  if (!std::isfinite(theta_next) || !std::isfinite(omega))
    return set_error(h, MNS_ERR_INVALID_ARG, "theta and omega must be finite");
  mns_step_opts o;
  mns_default_step_opts(&o);
  if (opts) o = *opts;
  if (!(o.newton_rtol >= 0) || !(o.newton_atol >= 0) || o.max_newton < 1 || o.max_newton > 100)
    return set_error(h, MNS_ERR_INVALID_ARG, "invalid step options");
  mns_step_report rep{};
  int rc;
  try {
    rc = mns_bdf2_step_impl(h, theta_next, omega, u_n, u_nm1, force, u_next, &o, &rep, as_stream(stream));
  } catch (...) {
    rc = set_error(h, MNS_ERR_HIP, "exception in time step");
  }
  if (report) *report = rep;
  return rc;
}

int mns_mg_levels(mns_handle* h, int* levels) {
  if (!h || !levels) return MNS_ERR_INVALID_ARG;
  if (!h->linearized) return set_error(h, MNS_ERR_NOT_LINEARIZED, "call mns_set_linearization first");
  try {
    return mns::mg_levels(h, levels, h->stream);
  } catch (...) {
    return set_error(h, MNS_ERR_HIP, "exception in mg_levels");
  }
}

int mns_mg_prolongate(mns_handle* h, int level, const double* x, double* y, void* stream) {
  if (!h) return MNS_ERR_INVALID_ARG;
  if (!h->linearized) return set_error(h, MNS_ERR_NOT_LINEARIZED, "call mns_set_linearization first");
  if (!aligned(x, 8) || !aligned(y, 8) || x == y)
    return set_error(h, MNS_ERR_INVALID_ARG, "x/y must be distinct 8-byte aligned pointers");
  try {
    return mns::mg_prolongate64(h, level, x, y, as_stream(stream));
  } catch (...) {
    return set_error(h, MNS_ERR_HIP, "exception in mg_prolongate");
  }
}

int mns_mg_restrict(mns_handle* h, int level, const double* x, double* y, void* stream) {
  if (!h) return MNS_ERR_INVALID_ARG;
  if (!h->linearized) return set_error(h, MNS_ERR_NOT_LINEARIZED, "call mns_set_linearization first");
  if (!aligned(x, 8) || !aligned(y, 8) || x == y)
    return set_error(h, MNS_ERR_INVALID_ARG, "x/y must be distinct 8-byte aligned pointers");
  try {
    return mns::mg_restrict64(h, level, x, y, as_stream(stream));
  } catch (...) {
    return set_error(h, MNS_ERR_HIP, "exception in mg_restrict");
  }
}

int mns_set_kernel_config(mns_handle* h, const mns_kernel_config* cfg) {
  if (!h || !cfg) return MNS_ERR_INVALID_ARG;
  if (cfg->fused_launch < -1 || cfg->fused_launch > 2)
    return set_error(h, MNS_ERR_INVALID_ARG, "fused_launch must be -1, 0, 1 or 2");
  if (cfg->volume_layout != 0 && cfg->volume_layout != 1)
    return set_error(h, MNS_ERR_INVALID_ARG, "volume_layout must be 0 or 1");
  if ((cfg->lin_source_f64 != 0 && cfg->lin_source_f64 != 1) || (cfg->lin_source_f32 != 0 && cfg->lin_source_f32 != 1))
    return set_error(h, MNS_ERR_INVALID_ARG, "lin_source_f64 and lin_source_f32 must be 0 or 1");
  h->fused = cfg->fused_launch;
  h->quad = cfg->volume_layout;
  h->lin_src[0] = cfg->lin_source_f64;
  h->lin_src[1] = cfg->lin_source_f32;
  return MNS_OK;
}

int mns_get_kernel_config(const mns_handle* h, mns_kernel_config* cfg) {
  if (!h || !cfg) return MNS_ERR_INVALID_ARG;
  cfg->fused_launch = h->fused;
  cfg->volume_layout = h->quad;
  cfg->lin_source_f64 = h->lin_src[0];
  cfg->lin_source_f32 = h->lin_src[1];
  return MNS_OK;
}

int mns_autotune_kernel_config(mns_handle* h, int reps, mns_kernel_config* chosen, void* stream) {
  if (!h || reps < 1 || reps > 1000) return MNS_ERR_INVALID_ARG;
  if (!h->linearized) return set_error(h, MNS_ERR_NOT_LINEARIZED, "call mns_set_linearization first");
  if (h->timing_cap) return set_error(h, MNS_ERR_INVALID_ARG, "disable kernel timing before autotuning");
  hipStream_t s = as_stream(stream);
  const size_t n = (size_t)h->ndofs;
  double *x = nullptr, *y = nullptr;
  float *x32 = nullptr, *y32 = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e;
  auto cleanup = [&]() {
    if (x) (void)hipFree(x);
    if (y) (void)hipFree(y);
    if (x32) (void)hipFree(x32);
    if (y32) (void)hipFree(y32);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  };
  if ((e = hipMalloc((void**)&x, n * sizeof(double))) != hipSuccess ||
      (e = hipMalloc((void**)&y, n * sizeof(double))) != hipSuccess ||
      (e = hipMalloc((void**)&x32, n * sizeof(float))) != hipSuccess ||
      (e = hipMalloc((void**)&y32, n * sizeof(float))) != hipSuccess ||
      (e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess) {
    cleanup();
    return set_error(h, MNS_ERR_HIP, std::string("autotune buffers: ") + hipGetErrorString(e));
  }
  int rc = mns::launch_fill<double>(x, 1.0, (int64_t)n, s);
  if (!rc) rc = mns::launch_fill<float>(x32, 1.0f, (int64_t)n, s);
  // milliseconds of `reps` applications in precision f32 with the current
  // configuration (two untimed first)
  auto time_apply = [&](bool f32, float* out) -> int {
    int r = MNS_OK;
    for (int i = 0; i < 2 + reps && r == MNS_OK; ++i) {
      if (i == 2) (void)hipEventRecord(e0, s);
      r = f32 ? mns::launch_jacobian<float>(h, x32, y32, s) : mns::launch_jacobian<double>(h, x, y, s);
    }
    (void)hipEventRecord(e1, s);
    if (r) return r;
    if ((e = hipEventSynchronize(e1)) != hipSuccess)
      return set_error(h, MNS_ERR_HIP, std::string("autotune sync: ") + hipGetErrorString(e));
    return hipEventElapsedTime(out, e0, e1) == hipSuccess ? MNS_OK : set_error(h, MNS_ERR_HIP, "autotune timing");
  };
  // candidates: every launch mode; both volume layouts where the quad layout
  // exists (3D, degrees 2 and 3); both linearization sources with the quad
  // layout where source C exists
  const bool has_quad = h->dim == 3 && (h->k == 2 || h->k == 3);
  const bool c64 = h->d_linc64 && h->k == 2, c32 = h->d_linc64 != nullptr;
  const mns_kernel_config saved{h->fused, h->quad, h->lin_src[0], h->lin_src[1]};
  float best = -1.0f;
  mns_kernel_config best_cfg = saved;
  for (int layout = has_quad ? 1 : saved.volume_layout; rc == MNS_OK && layout >= (has_quad ? 0 : saved.volume_layout);
       --layout)
    for (int mode = 0; rc == MNS_OK && mode <= 2; ++mode)
      for (int src = 0; rc == MNS_OK && src <= ((layout == 1 && c64) ? 1 : 0); ++src) {
        h->fused = mode;
        h->quad = layout;
        h->lin_src[0] = src;
        float ms = 0;
        if ((rc = time_apply(false, &ms))) break;
        if (best < 0 || ms < best) {
          best = ms;
          best_cfg.fused_launch = mode;
          best_cfg.volume_layout = layout;
          best_cfg.lin_source_f64 = src;
        }
      }
  // FP32 source with the chosen launch mode and layout
  if (rc == MNS_OK && c32 && best_cfg.volume_layout == 1) {
    h->fused = best_cfg.fused_launch;
    h->quad = best_cfg.volume_layout;
    float best32 = -1.0f;
    for (int src = 0; rc == MNS_OK && src <= 1; ++src) {
      h->lin_src[1] = src;
      float ms = 0;
      if ((rc = time_apply(true, &ms))) break;
      if (best32 < 0 || ms < best32) {
        best32 = ms;
        best_cfg.lin_source_f32 = src;
      }
    }
  }
  cleanup();
  if (rc) {
    h->fused = saved.fused_launch;
    h->quad = saved.volume_layout;
    h->lin_src[0] = saved.lin_source_f64;
    h->lin_src[1] = saved.lin_source_f32;
    return rc;
  }
  h->fused = best_cfg.fused_launch;
  h->quad = best_cfg.volume_layout;
  h->lin_src[0] = best_cfg.lin_source_f64;
  h->lin_src[1] = best_cfg.lin_source_f32;
  if (chosen) *chosen = best_cfg;
  return MNS_OK;
}

int mns_enable_timing(mns_handle* h, int capacity) {
  if (!h || capacity < 0) return MNS_ERR_INVALID_ARG;
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return set_error(h, MNS_ERR_HIP, std::string("sync: ") + hipGetErrorString(e));
  free_events(h);
  for (int c = 0; c < 3; ++c) {
    h->ev[c].resize(2 * (size_t)capacity);
    for (int i = 0; i < 2 * capacity; ++i)
      if ((e = hipEventCreate(&h->ev[c][i])) != hipSuccess) {
        h->ev[c].resize(i);
        free_events(h);
        return set_error(h, MNS_ERR_HIP, std::string("hipEventCreate: ") + hipGetErrorString(e));
      }
  }
  h->timing_cap = capacity;
  return MNS_OK;
}

int mns_read_timing(mns_handle* h, mns_timing* out) {
  if (!h || !out) return MNS_ERR_INVALID_ARG;
  double ms[3] = {0, 0, 0};
  for (int c = 0; c < 3; ++c)
    for (int i = 0; i < h->ev_used[c]; ++i) {
      hipError_t e = hipEventSynchronize(h->ev[c][2 * i + 1]);
      float t = 0;
      if (e == hipSuccess) e = hipEventElapsedTime(&t, h->ev[c][2 * i], h->ev[c][2 * i + 1]);
      if (e != hipSuccess) return set_error(h, MNS_ERR_HIP, std::string("event: ") + hipGetErrorString(e));
      ms[c] += t;
    }
  out->ms_volume = ms[0];
  out->ms_mortar = ms[1];
  out->ms_other = ms[2];
  out->n_volume = h->ev_used[0];
  out->n_mortar = h->ev_used[1];
  out->n_other = h->ev_used[2];
  for (int c = 0; c < 3; ++c) h->ev_used[c] = 0;
  return MNS_OK;
}

const char* mns_last_error(const mns_handle* h) { return h ? h->err.c_str() : "null handle"; }

void mns_destroy(mns_handle* h) {
  if (!h) return;
  if (h->d_cons) {  // the handle reached the device: drain its work first
    if (h->stream && !h->aux) (void)hipStreamSynchronize(h->stream);
    else (void)hipDeviceSynchronize();
  }
  free_all(h);
  delete h;
}

}  // extern "C"
