"""ctypes binding of libmortarns.so (C-ABI in include/mortarns.h).

Argument marshalling only: every computation runs in the HIP library.  Device
vectors are torch tensors (contiguous, float64 or float32, on the current HIP
device); their data pointers and torch's current stream are handed to the
library.  If the library is missing, `lib()` raises: there is no fallback.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmortarns.so")

MNS_OK = 0
MNS_ERR_INVALID_ARG = -1
MNS_ERR_HIP = -2
MNS_ERR_NOT_LINEARIZED = -3
MNS_ERR_NOT_CONVERGED = -4
MNS_ERR_UNSUPPORTED = -5
MNS_ERR_NO_ROTATION = -6
MNS_F64 = 0
MNS_F32 = 1
MNS_PRECOND_MG = 2
MNS_PRECOND_MG64 = 3
_PRECOND = {"none": -1, "f64": MNS_F64, "f32": MNS_F32, "mg": MNS_PRECOND_MG, "mg64": MNS_PRECOND_MG64}
MNS_LIN_NEWTON = 0
MNS_LIN_PICARD = 1
_LIN = {"newton": MNS_LIN_NEWTON, "picard": MNS_LIN_PICARD}

EXPORTED = [
    "mns_setup_mesh", "mns_n_dofs", "mns_rotate_rotor", "mns_set_linearization", "mns_apply_jacobian",
    "mns_apply_residual", "mns_compute_diagonal", "mns_default_solve_opts", "mns_solve", "mns_enable_timing",
    "mns_read_timing", "mns_set_kernel_config", "mns_get_kernel_config", "mns_last_error", "mns_destroy",
    "mns_default_step_opts", "mns_bdf2_step", "mns_mg_levels", "mns_mg_prolongate", "mns_set_linearization_kind",
    "mns_batch_create", "mns_batch_n_dofs", "mns_batch_apply_jacobian", "mns_batch_last_error", "mns_batch_destroy",
    "mns_autotune_kernel_config", "mns_mg_restrict", "mns_batch_solve", "mns_apply_jacobian_noalloc",
    "mns_assemble_matrix", "mns_stream_bandwidth", "mns_set_node_positions",
]


class MeshDesc(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int), ("degree", ctypes.c_int),
        ("r_in", ctypes.c_double), ("r_interface", ctypes.c_double), ("r_out", ctypes.c_double),
        ("height", ctypes.c_double),
        ("n_theta", ctypes.c_int), ("n_r_rotor", ctypes.c_int), ("n_r_stator", ctypes.c_int), ("n_z", ctypes.c_int),
        ("nu", ctypes.c_double), ("penalty_F", ctypes.c_double), ("penalty_side_rule", ctypes.c_int),
        ("steady", ctypes.c_int), ("dt", ctypes.c_double), ("n_theta_stator", ctypes.c_int),
    ]


class SolveOpts(ctypes.Structure):
    _fields_ = [
        ("rtol", ctypes.c_double), ("restart", ctypes.c_int), ("maxit", ctypes.c_int), ("precond", ctypes.c_int),
        ("cheb_degree", ctypes.c_int), ("cheb_range", ctypes.c_double), ("eig_iters", ctypes.c_int),
        ("mg_levels", ctypes.c_int), ("mg_smooth_degree", ctypes.c_int), ("mg_smooth_range", ctypes.c_double),
        ("mg_coarse_degree", ctypes.c_int), ("mg_coarse_linearization", ctypes.c_int),
        ("mg_fine_linearization", ctypes.c_int), ("use_graph", ctypes.c_int),
        ("cheb_lambda_factor", ctypes.c_double), ("mg_coarse_direct", ctypes.c_int),
    ]


def _set_fields(struct, opts):
    """Set ctypes fields by name; unknown names are errors (a plain setattr
    would add a Python attribute that the library never sees)."""
    names = {f for f, _ in struct._fields_}
    for k, v in opts.items():
        if k not in names:
            raise TypeError(f"unknown option {k!r} for {type(struct).__name__}")
        if k == "precond" and isinstance(v, str):
            v = _PRECOND[v]
        if k in ("mg_coarse_linearization", "mg_fine_linearization") and isinstance(v, str):
            v = _LIN[v]
        setattr(struct, k, v)


class SolveReport(ctypes.Structure):
    _fields_ = [
        ("iterations", ctypes.c_int), ("restarts", ctypes.c_int), ("status", ctypes.c_int),
        ("rel_residual", ctypes.c_double), ("lambda_max", ctypes.c_double), ("seconds", ctypes.c_double),
        ("vmults_f64", ctypes.c_int), ("vmults_f32", ctypes.c_int),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class StepOpts(ctypes.Structure):
    _fields_ = [
        ("newton_rtol", ctypes.c_double), ("newton_atol", ctypes.c_double), ("max_newton", ctypes.c_int),
        ("linear", SolveOpts),
    ]


class StepReport(ctypes.Structure):
    _fields_ = [
        ("newton_iterations", ctypes.c_int), ("linear_iterations", ctypes.c_int), ("status", ctypes.c_int),
        ("residual0", ctypes.c_double), ("residual", ctypes.c_double), ("seconds", ctypes.c_double),
        ("line_search_halvings", ctypes.c_int),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class KernelConfig(ctypes.Structure):
    _fields_ = [("fused_launch", ctypes.c_int), ("volume_layout", ctypes.c_int), ("lin_source_f64", ctypes.c_int),
                ("lin_source_f32", ctypes.c_int)]


class Timing(ctypes.Structure):
    _fields_ = [
        ("ms_volume", ctypes.c_double), ("ms_mortar", ctypes.c_double), ("ms_other", ctypes.c_double),
        ("n_volume", ctypes.c_int), ("n_mortar", ctypes.c_int), ("n_other", ctypes.c_int),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    """Load libmortarns.so; raises FileNotFoundError when it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise FileNotFoundError(f"{LIB_PATH} is missing: build it with paper_2608_27423_amd/build_lib.py")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64p = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)
        L.mns_setup_mesh.argtypes = [ctypes.POINTER(MeshDesc), vp, ctypes.POINTER(vp)]
        L.mns_n_dofs.argtypes = [vp, i64p, i64p]
        L.mns_rotate_rotor.argtypes = [vp, ctypes.c_double, ctypes.c_double, vp]
        L.mns_set_linearization.argtypes = [vp, vp, vp, vp, vp]
        L.mns_set_linearization_kind.argtypes = [vp, ctypes.c_int]
        L.mns_set_node_positions.argtypes = [vp, vp, ctypes.c_int64, vp]
        L.mns_apply_jacobian.argtypes = [vp, ctypes.c_int, vp, vp, vp]
        L.mns_apply_jacobian_noalloc.argtypes = [vp, ctypes.c_int, vp, vp, vp]
        L.mns_apply_residual.argtypes = [vp, vp, vp, vp]
        L.mns_assemble_matrix.argtypes = [vp, vp, ctypes.c_int64, vp]
        L.mns_stream_bandwidth.argtypes = [vp, vp, ctypes.c_int64, ctypes.c_int, ctypes.c_int, vp,
                                           ctypes.POINTER(ctypes.c_double)]
        L.mns_compute_diagonal.argtypes = [vp, ctypes.c_int, vp, vp]
        L.mns_default_solve_opts.argtypes = [ctypes.POINTER(SolveOpts)]
        L.mns_default_solve_opts.restype = None
        L.mns_solve.argtypes = [vp, vp, vp, ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveReport), vp]
        L.mns_enable_timing.argtypes = [vp, ctypes.c_int]
        L.mns_read_timing.argtypes = [vp, ctypes.POINTER(Timing)]
        L.mns_set_kernel_config.argtypes = [vp, ctypes.POINTER(KernelConfig)]
        L.mns_get_kernel_config.argtypes = [vp, ctypes.POINTER(KernelConfig)]
        L.mns_autotune_kernel_config.argtypes = [vp, ctypes.c_int, ctypes.POINTER(KernelConfig), vp]
        L.mns_default_step_opts.argtypes = [ctypes.POINTER(StepOpts)]
        L.mns_default_step_opts.restype = None
        L.mns_bdf2_step.argtypes = [vp, ctypes.c_double, ctypes.c_double, vp, vp, vp, vp, ctypes.POINTER(StepOpts),
                                    ctypes.POINTER(StepReport), vp]
        L.mns_mg_levels.argtypes = [vp, ctypes.POINTER(ctypes.c_int)]
        L.mns_mg_prolongate.argtypes = [vp, ctypes.c_int, vp, vp, vp]
        L.mns_mg_restrict.argtypes = [vp, ctypes.c_int, vp, vp, vp]
        L.mns_batch_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int, ctypes.POINTER(vp)]
        L.mns_batch_n_dofs.argtypes = [vp, i64p]
        L.mns_batch_apply_jacobian.argtypes = [vp, ctypes.c_int, vp, vp, vp]
        L.mns_batch_last_error.argtypes = [vp]
        L.mns_batch_last_error.restype = ctypes.c_char_p
        L.mns_batch_destroy.argtypes = [vp]
        L.mns_batch_solve.argtypes = [vp, vp, vp, ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveReport), vp]
        L.mns_batch_destroy.restype = None
        L.mns_last_error.argtypes = [vp]
        L.mns_last_error.restype = ctypes.c_char_p
        L.mns_destroy.argtypes = [vp]
        L.mns_destroy.restype = None
        _lib = L
    return _lib


def stream_bandwidth(read_bytes=1 << 31, ratio=6, reps=20):
    """GB/s of the library's read-dominated stream kernel (mns_stream_bandwidth)
    over device buffers allocated here."""
    import torch

    src = torch.ones(read_bytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty(read_bytes // 8 // max(int(ratio), 1) + 4, dtype=torch.float64, device="cuda")
    g = ctypes.c_double()
    rc = lib().mns_stream_bandwidth(_ptr(src), _ptr(dst), int(read_bytes), int(ratio), int(reps), _stream(),
                                    ctypes.byref(g))
    del src, dst
    torch.cuda.empty_cache()
    if rc != MNS_OK:
        raise MnsError(rc, "stream bandwidth")
    return g.value


class MnsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libmortarns error {code}: {msg}")
        self.code = code


def mesh_desc(mesh):
    """MeshDesc from a workload dictionary (see inputs.WORKLOADS)."""
    return MeshDesc(
        dim=int(mesh["dim"]), degree=int(mesh["degree"]), r_in=float(mesh["r_in"]),
        r_interface=float(mesh["r_if"]), r_out=float(mesh["r_out"]), height=float(mesh.get("height", 1.0)),
        n_theta=int(mesh["n_theta"]), n_r_rotor=int(mesh["n_r_rotor"]), n_r_stator=int(mesh["n_r_stator"]),
        n_z=int(mesh.get("n_z", 1)), nu=float(mesh["nu"]), penalty_F=float(mesh.get("penalty_F", 1.0)),
        penalty_side_rule=int(mesh.get("penalty_rule", 0)), steady=int(mesh.get("steady", 1)),
        dt=float(mesh.get("dt", 1.0)), n_theta_stator=int(mesh.get("n_theta_stator", 0)),
    )


def _stream():
    import torch

    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("vectors must be contiguous device tensors")
    return ctypes.c_void_p(t.data_ptr())


class Operator:
    """Handle around one rotor/stator problem (one mns_handle)."""

    def __init__(self, mesh):
        self._L = lib()
        self._h = ctypes.c_void_p()
        self.mesh = dict(mesh)
        desc = mesh_desc(mesh)
        rc = self._L.mns_setup_mesh(ctypes.byref(desc), _stream(), ctypes.byref(self._h))
        if rc != MNS_OK:
            msg = self.last_error()
            self.close()
            raise MnsError(rc, msg)
        a, b = ctypes.c_int64(), ctypes.c_int64()
        self._check(self._L.mns_n_dofs(self._h, ctypes.byref(a), ctypes.byref(b)))
        self.n_dofs, self.n_rotor = a.value, b.value

    def last_error(self):
        if not self._h:
            return ""
        return self._L.mns_last_error(self._h).decode()

    def _check(self, rc):
        if rc != MNS_OK:
            raise MnsError(rc, self.last_error())
        return rc

    def rotate_rotor(self, theta, omega):
        return self._check(self._L.mns_rotate_rotor(self._h, float(theta), float(omega), _stream()))

    def set_node_positions(self, xyz):
        """Iso-parametric geometry from node positions (host array, n_nodes x 3,
        rotor nodes in the material frame); None returns to the polar geometry
        (mns_set_node_positions).  Clears rotation and linearization."""
        import numpy as np

        if xyz is None:
            return self._check(self._L.mns_set_node_positions(self._h, None, 0, _stream()))
        a = np.ascontiguousarray(xyz, dtype=np.float64)
        if a.ndim != 2 or a.shape[1] != 3:
            raise ValueError("node positions must be an (n_nodes, 3) array")
        self._xyz = a
        return self._check(self._L.mns_set_node_positions(self._h, ctypes.c_void_p(a.ctypes.data), a.shape[0],
                                                          _stream()))

    def set_linearization(self, state, hist=None, force=None, kind=None):
        """kind: None (keep), "newton" or "picard" (mns_set_linearization_kind)."""
        if kind is not None:
            self._check(self._L.mns_set_linearization_kind(self._h, _LIN[kind] if isinstance(kind, str) else kind))
        self._keep = (state, hist, force)
        return self._check(self._L.mns_set_linearization(self._h, _ptr(state), _ptr(hist), _ptr(force), _stream()))

    def apply_jacobian(self, src, dst=None):
        import torch

        if dst is None:
            dst = torch.empty_like(src)
        prec = MNS_F64 if src.dtype == torch.float64 else MNS_F32
        if src.dtype not in (torch.float64, torch.float32) or dst.dtype != src.dtype:
            raise ValueError("src/dst must both be float64 or both float32")
        if src.numel() != self.n_dofs or dst.numel() != self.n_dofs:
            raise ValueError("vector length != n_dofs")
        self._check(self._L.mns_apply_jacobian(self._h, prec, _ptr(src), _ptr(dst), _stream()))
        return dst

    def apply_jacobian_noalloc(self, src, dst):
        """dst = J src through the allocation-free entry point (local results
        in the library's scratch array); dst must be given."""
        import torch

        prec = MNS_F64 if src.dtype == torch.float64 else MNS_F32
        if src.dtype not in (torch.float64, torch.float32) or dst.dtype != src.dtype:
            raise ValueError("src/dst must both be float64 or both float32")
        if src.numel() != self.n_dofs or dst.numel() != self.n_dofs:
            raise ValueError("vector length != n_dofs")
        self._check(self._L.mns_apply_jacobian_noalloc(self._h, prec, _ptr(src), _ptr(dst), _stream()))
        return dst

    def assemble_matrix(self):
        """Dense Jacobian (n x n, float64 tensor, row-major view of the
        column-major device matrix transposed back) by mns_assemble_matrix."""
        import torch

        A = torch.empty((self.n_dofs, self.n_dofs), dtype=torch.float64, device="cuda")
        self._check(self._L.mns_assemble_matrix(self._h, _ptr(A), self.n_dofs, _stream()))
        return A.t()  # column-major storage: A_cm[col][row]

    def apply_residual(self, state, res=None):
        import torch

        if res is None:
            res = torch.empty_like(state)
        if state.dtype != torch.float64 or state.numel() != self.n_dofs:
            raise ValueError("state must be float64 of length n_dofs")
        self._check(self._L.mns_apply_residual(self._h, _ptr(state), _ptr(res), _stream()))
        return res

    def compute_diagonal(self, dtype=None, out=None):
        import torch

        dtype = dtype or torch.float64
        if out is None:
            out = torch.empty(self.n_dofs, dtype=dtype, device="cuda")
        prec = MNS_F64 if out.dtype == torch.float64 else MNS_F32
        self._check(self._L.mns_compute_diagonal(self._h, prec, _ptr(out), _stream()))
        return out

    @staticmethod
    def default_solve_opts():
        o = SolveOpts()
        lib().mns_default_solve_opts(ctypes.byref(o))
        return o

    def solve(self, rhs, x=None, check=True, **opts):
        """FGMRES(FP64) with a Jacobi-Chebyshev preconditioner; returns (x, report dict)."""
        import torch

        o = self.default_solve_opts()
        _set_fields(o, opts)
        if x is None:
            x = torch.zeros_like(rhs)
        rep = SolveReport()
        rc = self._L.mns_solve(self._h, _ptr(rhs), _ptr(x), ctypes.byref(o), ctypes.byref(rep), _stream())
        if check and rc not in (MNS_OK,):
            raise MnsError(rc, self.last_error())
        d = rep.as_dict()
        d["rc"] = rc
        return x, d

    def bdf2_step(self, theta_next, omega, u_n, u_next, u_nm1=None, force=None, check=True, linear=None, **opts):
        """One BDF2 + Newton time step (mns_bdf2_step); u_next holds the initial
        guess and receives the solution.  Returns the report as a dict."""
        o = StepOpts()
        self._L.mns_default_step_opts(ctypes.byref(o))
        _set_fields(o, opts)
        _set_fields(o.linear, linear or {})
        for t in (u_n, u_next, u_nm1, force):
            if t is not None and (t.numel() != self.n_dofs or t.dtype.itemsize != 8):
                raise ValueError("vectors must be float64 of length n_dofs")
        rep = StepReport()
        rc = self._L.mns_bdf2_step(self._h, float(theta_next), float(omega), _ptr(u_n), _ptr(u_nm1), _ptr(force),
                                   _ptr(u_next), ctypes.byref(o), ctypes.byref(rep), _stream())
        if check and rc != MNS_OK:
            raise MnsError(rc, self.last_error())
        d = rep.as_dict()
        d["rc"] = rc
        return d

    def mg_levels(self):
        n = ctypes.c_int()
        self._check(self._L.mns_mg_levels(self._h, ctypes.byref(n)))
        return n.value

    def mg_prolongate(self, level, x, y):
        """y = P x from multigrid level `level`+1 to `level` (FP64 device vectors)."""
        return self._check(self._L.mns_mg_prolongate(self._h, int(level), _ptr(x), _ptr(y), _stream()))

    def mg_restrict(self, level, x, y):
        """y = P^T x from multigrid level `level` to `level`+1 (FP64 device vectors)."""
        return self._check(self._L.mns_mg_restrict(self._h, int(level), _ptr(x), _ptr(y), _stream()))

    def set_kernel_config(self, **kw):
        c = KernelConfig()
        self._check(self._L.mns_get_kernel_config(self._h, ctypes.byref(c)))
        names = {f for f, _ in KernelConfig._fields_}
        for k2, v in kw.items():
            if k2 not in names:
                raise TypeError(f"unknown kernel configuration field {k2!r}")
            setattr(c, k2, int(v))
        return self._check(self._L.mns_set_kernel_config(self._h, ctypes.byref(c)))

    def autotune_kernel_config(self, reps=10):
        """Time every launch configuration on this mesh and keep the fastest."""
        c = KernelConfig()
        self._check(self._L.mns_autotune_kernel_config(self._h, int(reps), ctypes.byref(c), _stream()))
        return {k2: getattr(c, k2) for k2, _ in c._fields_}

    def get_kernel_config(self):
        c = KernelConfig()
        self._check(self._L.mns_get_kernel_config(self._h, ctypes.byref(c)))
        return {k2: getattr(c, k2) for k2, _ in c._fields_}

    def enable_timing(self, capacity):
        return self._check(self._L.mns_enable_timing(self._h, int(capacity)))

    def read_timing(self):
        t = Timing()
        self._check(self._L.mns_read_timing(self._h, ctypes.byref(t)))
        return t.as_dict()

    def close(self):
        if getattr(self, "_h", None):
            self._L.mns_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


class Batch:
    """Instances of one dimension and degree applied together (mns_batch_*).
    Vectors are the instances' vectors concatenated in the order of `ops`;
    `offsets[i]` is where instance i starts."""

    def __init__(self, ops):
        self._L = lib()
        self._ops = list(ops)  # the handles must outlive the batch
        arr = (ctypes.c_void_p * len(self._ops))(*[op._h.value for op in self._ops])
        self._b = ctypes.c_void_p()
        rc = self._L.mns_batch_create(arr, len(self._ops), ctypes.byref(self._b))
        if rc != MNS_OK:
            raise MnsError(rc, self._ops[0].last_error() if self._ops else "")
        n = ctypes.c_int64()
        self._check(self._L.mns_batch_n_dofs(self._b, ctypes.byref(n)))
        self.n_dofs = n.value
        self.offsets = []
        off = 0
        for op in self._ops:
            self.offsets.append(off)
            off += op.n_dofs

    def _check(self, rc):
        if rc != MNS_OK:
            raise MnsError(rc, self.last_error())
        return rc

    def last_error(self):
        """Message of the batch's last failed call (mns_batch_last_error)."""
        return self._L.mns_batch_last_error(self._b).decode()

    def apply_jacobian(self, src, dst=None):
        import torch

        if dst is None:
            dst = torch.empty_like(src)
        prec = MNS_F64 if src.dtype == torch.float64 else MNS_F32
        if src.dtype not in (torch.float64, torch.float32) or dst.dtype != src.dtype:
            raise ValueError("src/dst must both be float64 or both float32")
        if src.numel() != self.n_dofs or dst.numel() != self.n_dofs:
            raise ValueError("vector length != batch n_dofs")
        self._check(self._L.mns_batch_apply_jacobian(self._b, prec, _ptr(src), _ptr(dst), _stream()))
        return dst

    def solve(self, rhs, x=None, check=True, **opts):
        """Batched FGMRES (mns_batch_solve); returns (x, rc, list of per-instance report dicts)."""
        import torch

        o = Operator.default_solve_opts()
        _set_fields(o, opts)
        if x is None:
            x = torch.zeros_like(rhs)
        if rhs.numel() != self.n_dofs or x.numel() != self.n_dofs:
            raise ValueError("vector length != batch n_dofs")
        reps = (SolveReport * len(self._ops))()
        rc = self._L.mns_batch_solve(self._b, _ptr(rhs), _ptr(x), ctypes.byref(o), reps, _stream())
        if check and rc != MNS_OK:
            raise MnsError(rc, self._L.mns_batch_last_error(self._b).decode())
        return x, rc, [r.as_dict() for r in reps]

    def close(self):
        if getattr(self, "_b", None):
            self._L.mns_batch_destroy(self._b)
            self._b = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
