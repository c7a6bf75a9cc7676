"""FP64 CPU oracle for the stabilized ALE Navier-Stokes Jacobian with mortar faces.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no code
with the HIP library in ``paper_2608_27423_amd`` and never imports it; the two
meet only through the seeded inputs of ``paper_2608_27423_amd.inputs``.

This module only marshals arrays to ``libmns_oracle.so`` (built from
``mns_oracle.c`` with gcc + OpenMP); every step of the arithmetic is in that C
file, which cites the paper passage each part follows.

Functions with no independent pin ("parity unpinned"): none of the operator
parts; the angle-insensitivity study of Sec. 4.1 has no printed values and is
only reported.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mns_oracle.c")
_LIB = os.path.join(_HERE, "libmns_oracle.so")
_lib = None


def build(force=True):
    """Compile the oracle with gcc (-O2, OpenMP).  Returns the library path."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fopenmp", "-fPIC", "-shared", _SRC, "-o", tmp, "-lm"]
        )
        os.replace(tmp, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int), ("degree", ctypes.c_int),
        ("r_in", ctypes.c_double), ("r_if", ctypes.c_double), ("r_out", ctypes.c_double),
        ("height", ctypes.c_double),
        ("n_theta", ctypes.c_int), ("n_r_rotor", ctypes.c_int), ("n_r_stator", ctypes.c_int),
        ("n_z", ctypes.c_int),
        ("nu", ctypes.c_double), ("penalty_F", ctypes.c_double),
        ("penalty_rule", ctypes.c_int), ("steady", ctypes.c_int), ("dt", ctypes.c_double),
        ("theta_rot", ctypes.c_double), ("omega", ctypes.c_double),
        ("merged", ctypes.c_int), ("stabilization", ctypes.c_int), ("pin_pressure", ctypes.c_int),
        ("mms", ctypes.c_int), ("nthreads", ctypes.c_int), ("picard", ctypes.c_int),
        ("n_theta_stator", ctypes.c_int), ("iso", ctypes.c_int), ("perturb", ctypes.c_double),
    ]


_DEFAULTS = dict(
    dim=2, degree=2, r_in=0.25, r_if=0.5, r_out=1.0, height=1.0, n_theta=8, n_r_rotor=1,
    n_r_stator=1, n_z=1, nu=0.01, penalty_F=1.0, penalty_rule=0, steady=1, dt=1.0, theta_rot=0.0,
    omega=0.0, merged=0, stabilization=1, pin_pressure=1, mms=0, nthreads=0, picard=0, n_theta_stator=0,
    iso=0, perturb=0.0,
)


def _configure(lib):
    P = ctypes.POINTER(_Params)
    dp = ctypes.POINTER(ctypes.c_double)
    i64p = ctypes.POINTER(ctypes.c_int64)
    lib.orc_ndofs.argtypes = [P, i64p, i64p, i64p, i64p]
    lib.orc_constrained.argtypes = [P, ctypes.c_void_p]
    lib.orc_node_coords.argtypes = [P, dp]
    lib.orc_cell_info.argtypes = [P, dp, dp, dp, dp]
    lib.orc_segments.argtypes = [P, ctypes.c_void_p, dp, dp]
    lib.orc_rules.argtypes = [ctypes.c_int, dp, dp, dp]
    lib.orc_lagrange.argtypes = [ctypes.c_int, dp, ctypes.c_double, dp, dp, dp]
    lib.orc_phys_basis.argtypes = [P, ctypes.c_int64, dp, dp, dp, dp, dp]
    lib.orc_apply_jacobian.argtypes = [P, dp, dp, dp, dp, dp]
    lib.orc_apply_jacobian_rows.argtypes = [P, dp, dp, dp, dp, ctypes.c_int64, i64p, dp]
    lib.orc_residual.argtypes = [P, dp, dp, dp, dp, dp]
    lib.orc_diagonal.argtypes = [P, dp, dp, dp, dp]
    lib.orc_assemble.argtypes = [P, dp, dp, dp, ctypes.c_int64, i64p, i64p, dp, i64p]
    lib.orc_mms_interpolate.argtypes = [P, dp]
    lib.orc_mms_errors.argtypes = [P, dp, dp]
    return lib


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = _configure(ctypes.CDLL(_LIB))
    return _lib


def build_variant(source_text, path):
    """Compile another version of the oracle source (the planted-mistake tests
    use this to check that the pins reject a wrong oracle)."""
    src = path + ".c"
    with open(src, "w") as f:
        f.write(source_text)
    subprocess.check_call(["gcc", "-O1", "-std=c11", "-D_GNU_SOURCE", "-fopenmp", "-fPIC", "-shared", src, "-o", path,
                           "-lm"])
    return path


def swap_library(path):
    """Route every oracle call to the library at `path` (None: the real
    oracle).  Returns the previously active library handle."""
    global _lib
    old = _lib
    _lib = None if path is None else _configure(ctypes.CDLL(path))
    return old


def params(**kw):
    """Oracle parameter set; unknown keys are rejected."""
    d = dict(_DEFAULTS)
    for k, v in kw.items():
        if k not in d:
            raise KeyError(f"unknown oracle parameter {k!r}")
        d[k] = v
    return d


def _struct(cfg):
    d = dict(_DEFAULTS)
    d.update({k: v for k, v in cfg.items() if k in _DEFAULTS})
    return _Params(**d)


def _dp(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a, n=None):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    if n is not None and a.shape != (n,):
        raise ValueError(f"expected shape ({n},), got {a.shape}")
    return a


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


def sizes(cfg):
    """(n_dofs, n_rotor_dofs, n_cells, n_segments)."""
    lib = _load()
    v = [ctypes.c_int64() for _ in range(4)]
    _check(lib.orc_ndofs(ctypes.byref(_struct(cfg)), *[ctypes.byref(x) for x in v]), "sizes")
    return tuple(int(x.value) for x in v)


def n_dofs(cfg):
    return sizes(cfg)[0]


def constrained(cfg):
    n = n_dofs(cfg)
    m = np.zeros(n, dtype=np.uint8)
    _check(_load().orc_constrained(ctypes.byref(_struct(cfg)), m.ctypes.data), "constrained")
    return m.astype(bool)


def node_coords(cfg):
    n = n_dofs(cfg) // (cfg["dim"] + 1)
    xyz = np.zeros((n, 3))
    _check(_load().orc_node_coords(ctypes.byref(_struct(cfg)), _dp(xyz)), "node_coords")
    return xyz


def cell_info(cfg):
    nc = sizes(cfg)[2]
    h, V, tp = np.zeros(nc), np.zeros(nc), np.zeros(nc)
    ts = np.zeros(2)
    _check(_load().orc_cell_info(ctypes.byref(_struct(cfg)), _dp(h), _dp(V), _dp(tp), _dp(ts)), "cell_info")
    return dict(h=h, V=V, tau_pen=tp, tau_side=ts)


def segments(cfg):
    ns = sizes(cfg)[3]
    n = cfg["degree"] + 1
    nqz = n if cfg["dim"] == 3 else 1
    ids = np.zeros((max(ns, 1), 3), dtype=np.int32)
    lohi = np.zeros((max(ns, 1), 2))
    jxw = np.zeros(max(ns, 1) * nqz * n)
    _check(_load().orc_segments(ctypes.byref(_struct(cfg)), ids.ctypes.data, _dp(lohi), _dp(jxw)), "segments")
    return ids[:ns], lohi[:ns], jxw[: ns * nqz * n]


def rules(n):
    gll, gx, gw = np.zeros(n), np.zeros(n), np.zeros(n)
    _check(_load().orc_rules(n, _dp(gll), _dp(gx), _dp(gw)), "rules")
    return gll, gx, gw


def lagrange(nodes, t):
    nodes = _f64(nodes)
    n = nodes.size
    L, dL, d2L = np.zeros(n), np.zeros(n), np.zeros(n)
    _check(_load().orc_lagrange(n, _dp(nodes), float(t), _dp(L), _dp(dL), _dp(d2L)), "lagrange")
    return L, dL, d2L


def phys_basis(cfg, cell, xi):
    n = cfg["degree"] + 1
    nd = n ** cfg["dim"]
    xi = _f64(list(xi) + [0.0] * (3 - len(xi)))
    phi, grad, lap, x = np.zeros(nd), np.zeros((nd, 3)), np.zeros(nd), np.zeros(3)
    _check(_load().orc_phys_basis(ctypes.byref(_struct(cfg)), int(cell), _dp(xi), _dp(phi), _dp(grad),
                                  _dp(lap), _dp(x)), "phys_basis")
    return phi, grad, lap, x


def apply_jacobian(cfg, state, x, hist=None, force=None):
    """y = J(state) x with constrained columns zero and constrained rows y = x."""
    n = n_dofs(cfg)
    state, x, hist, force = _f64(state, n), _f64(x, n), _f64(hist, n), _f64(force, n)
    y = np.zeros(n)
    _check(_load().orc_apply_jacobian(ctypes.byref(_struct(cfg)), _dp(state), _dp(hist), _dp(force), _dp(x),
                                      _dp(y)), "apply_jacobian")
    return y


def apply_jacobian_rows(cfg, state, x, rows, hist=None, force=None):
    n = n_dofs(cfg)
    state, x, hist, force = _f64(state, n), _f64(x, n), _f64(hist, n), _f64(force, n)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    out = np.zeros(rows.size)
    _check(_load().orc_apply_jacobian_rows(ctypes.byref(_struct(cfg)), _dp(state), _dp(hist), _dp(force),
                                           _dp(x), rows.size,
                                           rows.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _dp(out)),
           "apply_jacobian_rows")
    return out


def residual(cfg, state, hist=None, force=None, tau_state=None):
    """Nonlinear residual; tau from ``tau_state`` when given (frozen)."""
    n = n_dofs(cfg)
    state, hist, force, tau_state = _f64(state, n), _f64(hist, n), _f64(force, n), _f64(tau_state, n)
    r = np.zeros(n)
    _check(_load().orc_residual(ctypes.byref(_struct(cfg)), _dp(state), _dp(hist), _dp(force), _dp(tau_state),
                                _dp(r)), "residual")
    return r


def diagonal(cfg, state, hist=None, force=None):
    n = n_dofs(cfg)
    state, hist, force = _f64(state, n), _f64(hist, n), _f64(force, n)
    dg = np.zeros(n)
    _check(_load().orc_diagonal(ctypes.byref(_struct(cfg)), _dp(state), _dp(hist), _dp(force), _dp(dg)),
           "diagonal")
    return dg


def assemble(cfg, state, hist=None, force=None):
    """Assembled constrained Jacobian as a scipy CSR matrix (tiny meshes)."""
    import scipy.sparse as sp

    lib = _load()
    n = n_dofs(cfg)
    state, hist, force = _f64(state, n), _f64(hist, n), _f64(force, n)
    cnt = ctypes.c_int64()
    P = _struct(cfg)
    _check(lib.orc_assemble(ctypes.byref(P), _dp(state), _dp(hist), _dp(force), 0, None, None, None,
                            ctypes.byref(cnt)), "assemble(size)")
    cap = cnt.value
    rows = np.zeros(cap, dtype=np.int64)
    cols = np.zeros(cap, dtype=np.int64)
    vals = np.zeros(cap)
    i64 = ctypes.POINTER(ctypes.c_int64)
    _check(lib.orc_assemble(ctypes.byref(P), _dp(state), _dp(hist), _dp(force), cap, rows.ctypes.data_as(i64),
                            cols.ctypes.data_as(i64), _dp(vals), ctypes.byref(cnt)), "assemble")
    k = cnt.value
    return sp.coo_matrix((vals[:k], (rows[:k], cols[:k])), shape=(n, n)).tocsr()


def mms_interpolate(cfg):
    v = np.zeros(n_dofs(cfg))
    _check(_load().orc_mms_interpolate(ctypes.byref(_struct(cfg)), _dp(v)), "mms_interpolate")
    return v


def mms_errors(cfg, sol):
    err = np.zeros(2)
    sol = _f64(sol, n_dofs(cfg))
    _check(_load().orc_mms_errors(ctypes.byref(_struct(cfg)), _dp(sol), _dp(err)), "mms_errors")
    return float(err[0]), float(err[1])
