"""GPU (HIP, gfx950) vs the FP64 oracle, element by element, through the C-ABI.

Bar: FP64 results match the oracle to a relative max-norm of 1e-12; the FP32
instance is reported and held to a loose sanity bound (it is a preconditioner
precision, not a parity claim).
"""
import math

import numpy as np
import pytest
import torch

import oracle
from helpers import oracle_cfg, relmax, small_mesh
from paper_2608_27423_amd import binding, inputs

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 5e-5


def _dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def _gpu_apply(mesh, theta, omega, state, x, hist=None, force=None, fused=-1, layout=1):
    with binding.Operator(mesh) as op:
        op.set_kernel_config(fused_launch=fused, volume_layout=layout)
        op.rotate_rotor(theta, omega)
        op.set_linearization(_dev(state), None if hist is None else _dev(hist),
                             None if force is None else _dev(force))
        y64 = op.apply_jacobian(_dev(x)).cpu().numpy()
        y32 = op.apply_jacobian(_dev(x, torch.float32)).double().cpu().numpy()
        torch.cuda.synchronize()
    return y64, y32


CASES = [(2, 2), (2, 3), (2, 4), (2, 5), (3, 2), (3, 3), (3, 4)]
# kernel configurations: (fused launch, volume layout)
KCONF = [(1, 1), (0, 1), (2, 1), (-1, 1), (1, 0), (0, 0), (2, 0)]


@pytest.mark.parametrize("dim,k", CASES)
@pytest.mark.parametrize("angle", ["random", "aligned", "near_aligned", "negative_wrapped"])
@pytest.mark.parametrize("fused,layout", KCONF)
def test_jacobian_small(dim, k, angle, fused, layout):
    mesh = small_mesh(dim, k)
    dth = 2 * math.pi / mesh["n_theta"]
    theta = {"random": 2.345, "aligned": 2 * dth, "near_aligned": 3 * dth - 1e-14,
             "negative_wrapped": -7.9}[angle]
    g = np.random.default_rng(100 * dim + k)
    n = inputs.n_dofs(mesh)
    state, x = g.uniform(-1, 1, n), g.uniform(-1, 1, n)
    y64, y32 = _gpu_apply(mesh, theta, 0.8, state, x, fused=fused, layout=layout)
    yo = oracle.apply_jacobian(oracle_cfg(mesh, theta, 0.8), state, x)
    e64, e32 = relmax(y64, yo), relmax(y32, yo)
    print(f"dim={dim} k={k} {angle} fused={fused} layout={layout}: fp64 {e64:.2e} fp32 {e32:.2e}")
    assert e64 <= TOL64
    assert e32 <= TOL32


@pytest.mark.parametrize("n_theta", [16, 32])
@pytest.mark.parametrize("angle", ["random", "aligned"])
@pytest.mark.parametrize("fused", [1, 0, 2])
def test_jacobian_strip_layout(n_theta, angle, fused):
    """3D Q2 with a ring length that is a multiple of 16: the quad kernel sums
    the shared theta faces of its 16 cells before storing (strip layout) and
    the gather reads that layout, including the batch-boundary columns and the
    periodic wrap."""
    mesh = small_mesh(3, 2, n_theta=n_theta)
    dth = 2 * math.pi / n_theta
    theta = {"random": 2.345, "aligned": 5 * dth}[angle]
    g = np.random.default_rng(300 + n_theta)
    n = inputs.n_dofs(mesh)
    state, x = g.uniform(-1, 1, n), g.uniform(-1, 1, n)
    y64, y32 = _gpu_apply(mesh, theta, 0.8, state, x, fused=fused, layout=1)
    yo = oracle.apply_jacobian(oracle_cfg(mesh, theta, 0.8), state, x)
    e64, e32 = relmax(y64, yo), relmax(y32, yo)
    print(f"strip n_theta={n_theta} {angle} fused={fused}: fp64 {e64:.2e} fp32 {e32:.2e}")
    assert e64 <= TOL64
    assert e32 <= TOL32


@pytest.mark.parametrize("dim", [2, 3])
def test_jacobian_transient_with_history_and_force(dim):
    mesh = small_mesh(dim, 2, steady=0, dt=0.05, penalty_rule=1, penalty_F=3.0, n_theta=7)
    g = np.random.default_rng(7 + dim)
    n = inputs.n_dofs(mesh)
    state, x, hist, force = (g.uniform(-1, 1, n) for _ in range(4))
    y64, _ = _gpu_apply(mesh, 1.1, -0.4, state, x, hist, force)
    yo = oracle.apply_jacobian(oracle_cfg(mesh, 1.1, -0.4), state, x, hist=hist, force=force)
    assert relmax(y64, yo) <= TOL64


@pytest.mark.parametrize("dim,k,steady", [(2, 2, 1), (2, 3, 0), (3, 2, 1), (3, 2, 0), (3, 3, 1)])
def test_picard_linearization(dim, k, steady):
    """MNS_LIN_PICARD against the oracle's Picard option (no reaction term, no
    SUPG weight derivative): Jacobian in FP64 and FP32, and the diagonal; then
    the handle switches back to the Newton linearization."""
    mesh = small_mesh(dim, k, steady=steady, dt=0.05)
    g = np.random.default_rng(40 + 10 * dim + k)
    n = inputs.n_dofs(mesh)
    state, x, hist, force = (g.uniform(-1, 1, n) for _ in range(4))
    hist = None if steady else hist
    cfg = oracle_cfg(mesh, 1.9, 0.7)
    with binding.Operator(mesh) as op:
        op.rotate_rotor(1.9, 0.7)
        op.set_linearization(_dev(state), None if hist is None else _dev(hist), _dev(force), kind="picard")
        y64 = op.apply_jacobian(_dev(x)).cpu().numpy()
        y32 = op.apply_jacobian(_dev(x, torch.float32)).double().cpu().numpy()
        d64 = op.compute_diagonal(torch.float64).cpu().numpy()
        op.set_linearization(_dev(state), None if hist is None else _dev(hist), _dev(force), kind="newton")
        yn = op.apply_jacobian(_dev(x)).cpu().numpy()
    yo = oracle.apply_jacobian(dict(cfg, picard=1), state, x, hist=hist, force=force)
    do = oracle.diagonal(dict(cfg, picard=1), state, hist=hist, force=force)
    yno = oracle.apply_jacobian(cfg, state, x, hist=hist, force=force)
    print(f"picard dim={dim} k={k} steady={steady}: fp64 {relmax(y64, yo):.2e} fp32 {relmax(y32, yo):.2e} "
          f"diag {relmax(d64, do):.2e}; newton after {relmax(yn, yno):.2e}")
    assert relmax(yo, yno) > 1e-3
    assert relmax(y64, yo) <= TOL64
    assert relmax(y32, yo) <= TOL32
    assert relmax(d64, do) <= TOL64
    assert relmax(yn, yno) <= TOL64


@pytest.mark.parametrize("dim,k", [(2, 2), (2, 3), (3, 2), (3, 3)])
def test_residual(dim, k):
    mesh = small_mesh(dim, k, steady=0, dt=0.1)
    g = np.random.default_rng(3 + k)
    n = inputs.n_dofs(mesh)
    state, hist, force = (g.uniform(-1, 1, n) for _ in range(3))
    with binding.Operator(mesh) as op:
        op.rotate_rotor(0.77, 1.3)
        op.set_linearization(_dev(state), _dev(hist), _dev(force))
        r = op.apply_residual(_dev(state)).cpu().numpy()
    ro = oracle.residual(oracle_cfg(mesh, 0.77, 1.3), state, hist, force)
    assert relmax(r, ro) <= TOL64


@pytest.mark.parametrize("dim,k", [(2, 2), (2, 4), (3, 2), (3, 3)])
def test_diagonal(dim, k):
    mesh = small_mesh(dim, k)
    g = np.random.default_rng(11)
    n = inputs.n_dofs(mesh)
    state = g.uniform(-1, 1, n)
    with binding.Operator(mesh) as op:
        op.rotate_rotor(0.4, 0.9)
        op.set_linearization(_dev(state))
        d64 = op.compute_diagonal(torch.float64).cpu().numpy()
        d32 = op.compute_diagonal(torch.float32).double().cpu().numpy()
    do = oracle.diagonal(oracle_cfg(mesh, 0.4, 0.9), state)
    assert relmax(d64, do) <= TOL64
    assert relmax(d32, do) <= TOL32


def test_degenerate_inputs():
    """Zero input gives zero output except constrained rows (= input); the
    minimum mesh (3 cells per ring, one radial cell) and a zero state."""
    mesh = small_mesh(3, 2, n_theta=3, n_r_rotor=1, n_r_stator=1, n_z=1)
    n = inputs.n_dofs(mesh)
    zero = np.zeros(n)
    y64, _ = _gpu_apply(mesh, 0.3, 0.0, zero, zero)
    assert np.all(y64 == 0)
    g = np.random.default_rng(2)
    x = g.uniform(-1, 1, n)
    y64, _ = _gpu_apply(mesh, 0.3, 0.0, zero, x)
    yo = oracle.apply_jacobian(oracle_cfg(mesh, 0.3, 0.0), zero, x)
    assert relmax(y64, yo) <= TOL64


def test_workload_2d_q2_full():
    name = "annulus2d_q2_32x4"
    mesh = inputs.mesh(name)
    theta = inputs.rotor_angle(name)
    state, x = inputs.state_for(name), inputs.vector_for(name)
    y64, y32 = _gpu_apply(mesh, theta, mesh["omega"], state, x)
    yo = oracle.apply_jacobian(oracle_cfg(mesh, theta, mesh["omega"]), state, x)
    print(f"{name}: fp64 {relmax(y64, yo):.2e} fp32 {relmax(y32, yo):.2e}")
    assert relmax(y64, yo) <= TOL64
    assert relmax(y32, yo) <= TOL32


@pytest.mark.parametrize("layout", [1, 0])
def test_workload_3d_q2_full(layout):
    name = "annulus3d_q2_64x8x32"
    mesh = inputs.mesh(name)
    theta = inputs.rotor_angle(name)
    state, x = inputs.state_for(name), inputs.vector_for(name)
    y64, y32 = _gpu_apply(mesh, theta, mesh["omega"], state, x, layout=layout)
    yo = oracle.apply_jacobian(oracle_cfg(mesh, theta, mesh["omega"]), state, x)
    print(f"{name} layout={layout}: fp64 {relmax(y64, yo):.2e} fp32 {relmax(y32, yo):.2e}")
    assert relmax(y64, yo) <= TOL64
    assert relmax(y32, yo) <= TOL32


@pytest.mark.parametrize("name", ["annulus3d_q3_64x16x32", "annulus3d_q2_256x32x128"])
def test_workload_large_full(name):
    """Degree-3 7.3M-DoF and degree-2 68M-DoF workloads: the whole FP64 and
    FP32 products against the oracle's full product (every row)."""
    import time

    mesh = inputs.mesh(name)
    theta = inputs.rotor_angle(name)
    state, x = inputs.state_for(name), inputs.vector_for(name)
    y64, y32 = _gpu_apply(mesh, theta, mesh["omega"], state, x)
    t0 = time.perf_counter()
    yo = oracle.apply_jacobian(oracle_cfg(mesh, theta, mesh["omega"]), state, x)
    t_or = time.perf_counter() - t0
    e64, e32 = relmax(y64, yo), relmax(y32, yo)
    print(f"{name}: {x.size} rows (oracle {t_or:.1f} s), fp64 {e64:.2e} fp32 {e32:.2e}", flush=True)
    assert e64 <= TOL64
    assert e32 <= TOL32


@pytest.mark.parametrize("precond", ["f64", "f32"])
def test_solve_2d_workload(precond):
    """FGMRES(FP64) with the Jacobi-Chebyshev preconditioner in FP64 or FP32
    reaches 1e-8; the true residual is recomputed with the oracle's operator."""
    name = "annulus2d_q2_32x4"
    mesh = inputs.mesh(name)
    theta = inputs.rotor_angle(name)
    st = inputs.state_for(name)
    st = st / np.abs(st).max()
    n = st.size
    xstar = inputs.uniform(n, inputs.SOLUTION_SEED[name])
    cfg = oracle_cfg(mesh, theta, mesh["omega"])
    b = oracle.apply_jacobian(cfg, st, xstar)
    with binding.Operator(mesh) as op:
        op.rotate_rotor(theta, mesh["omega"])
        op.set_linearization(_dev(st))
        x, info = op.solve(_dev(b), restart=250, maxit=2000, precond=precond, cheb_degree=4)
        x = x.cpu().numpy()
    r = b - oracle.apply_jacobian(cfg, st, x)
    rel = np.linalg.norm(r) / np.linalg.norm(b)
    print(f"solve {precond}: {info['iterations']} its, {info['seconds']:.3f}s, reported {info['rel_residual']:.2e},"
          f" oracle {rel:.2e}")
    assert info["rc"] == 0
    assert rel <= 1.01e-8


def test_chebyshev_interval_factor():
    """mns_solve_opts.cheb_lambda_factor widens the top of the Chebyshev
    interval: the reported lambda_max (the power-iteration estimate) does not
    depend on it, both settings reach 1e-8 against the oracle's operator, and
    factors outside [1, 4] are rejected."""
    name = "annulus2d_q2_32x4"
    mesh = inputs.mesh(name)
    theta = inputs.rotor_angle(name)
    st = inputs.state_for(name)
    st = st / np.abs(st).max()
    n = st.size
    cfg = oracle_cfg(mesh, theta, mesh["omega"])
    b = oracle.apply_jacobian(cfg, st, inputs.uniform(n, inputs.SOLUTION_SEED[name]))
    reps = {}
    with binding.Operator(mesh) as op:
        op.rotate_rotor(theta, mesh["omega"])
        op.set_linearization(_dev(st))
        for fac in (1.0, 1.05, 1.3):
            x, info = op.solve(_dev(b), restart=250, maxit=2000, precond="f32", cheb_degree=4,
                               cheb_lambda_factor=fac)
            r = b - oracle.apply_jacobian(cfg, st, x.cpu().numpy())
            assert info["rc"] == 0 and np.linalg.norm(r) <= 1.01e-8 * np.linalg.norm(b)
            reps[fac] = info
        for bad in (0.99, 4.5):
            _, info = op.solve(_dev(b), check=False, cheb_lambda_factor=bad)
            assert info["rc"] == binding.MNS_ERR_INVALID_ARG
        with pytest.raises(TypeError):
            op.solve(_dev(b), cheb_lambda_fact=1.1)
    print({f: (i["iterations"], i["lambda_max"]) for f, i in reps.items()})
    assert reps[1.0]["lambda_max"] == reps[1.05]["lambda_max"] == reps[1.3]["lambda_max"]
    assert reps[1.0]["iterations"] != reps[1.3]["iterations"]


@pytest.mark.parametrize("dim,k", [(2, 2), (3, 2), (3, 3)])
def test_autotune_keeps_parity(dim, k):
    """mns_autotune_kernel_config picks one of the launch configurations, sets
    it on the handle, and the product is unchanged (oracle parity)."""
    mesh = small_mesh(dim, k, n_theta=16)
    g = np.random.default_rng(60 + dim + k)
    n = inputs.n_dofs(mesh)
    state, x = g.uniform(-1, 1, n), g.uniform(-1, 1, n)
    with binding.Operator(mesh) as op:
        with pytest.raises(binding.MnsError):
            op.autotune_kernel_config(3)
        op.rotate_rotor(1.3, 0.6)
        op.set_linearization(_dev(state))
        chosen = op.autotune_kernel_config(5)
        assert chosen == op.get_kernel_config()
        assert chosen["fused_launch"] in (0, 1, 2)
        if dim == 2:
            assert chosen["volume_layout"] == 1  # unchanged where only one layout exists
        y = op.apply_jacobian(_dev(x)).cpu().numpy()
    yo = oracle.apply_jacobian(oracle_cfg(mesh, 1.3, 0.6), state, x)
    print(f"autotune dim={dim} k={k}: {chosen}, fp64 {relmax(y, yo):.2e}")
    assert relmax(y, yo) <= TOL64
