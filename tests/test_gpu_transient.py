"""GPU time step (BDF2 + Newton, mns_bdf2_step) against Newton's method on the
oracle: both must reach the same root of the discrete residual.

The oracle side assembles the Jacobian (tau frozen at the iterate) and solves
each Newton step directly with scipy; the GPU side uses the matrix-free
operator and FGMRES with the Jacobi-Chebyshev preconditioner.
"""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle
from paper_2608_27423_amd import binding, inputs
from tests.helpers import oracle_cfg, relmax, small_mesh

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=torch.float64)


def _oracle_step(cfg, un, unm1, force, guess, dt, rtol=1e-12, maxit=30):
    hist = (unm1 - 4.0 * un) / (2.0 * dt) if unm1 is not None else -3.0 * un / (2.0 * dt)
    u = guess.copy()
    r0 = None
    for _ in range(maxit):
        r = oracle.residual(cfg, u, hist, force)
        rn = np.linalg.norm(r)
        r0 = rn if r0 is None else r0
        if rn <= rtol * r0:
            return u, rn
        A = oracle.assemble(cfg, u, hist, force).tocsc()
        u = u + spla.spsolve(A, -r)
    raise AssertionError("oracle Newton did not converge")


def _start_fields(mesh, seed):
    """Two previous time levels: small smooth-ish fields with the Dirichlet
    values (zero on the walls, zero at the pinned pressure node)."""
    g = np.random.default_rng(seed)
    n = inputs.n_dofs(mesh)
    cfg = oracle_cfg(mesh, 0.0, 0.0)
    cons = oracle.constrained(cfg).astype(bool)
    un = 0.3 * g.uniform(-1, 1, n)
    unm1 = un + 0.02 * g.uniform(-1, 1, n)
    f = 0.5 * g.uniform(-1, 1, n)
    for v in (un, unm1):
        v[cons] = 0.0
    return un, unm1, f


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("first_step", [False, True])
def test_bdf2_step_matches_oracle_newton(dim, first_step):
    dt = 0.05
    mesh = small_mesh(dim, 2, n_theta=8 if dim == 2 else 5, steady=0, dt=dt, nu=0.02)
    un, unm1, f = _start_fields(mesh, 40 + dim)
    if first_step:
        unm1 = None
    theta, omega = 0.73, 0.6
    cfg = oracle_cfg(mesh, theta, omega)
    uo, _ = _oracle_step(cfg, un, unm1, f, un, dt)
    with binding.Operator(mesh) as op:
        u = _dev(un).clone()
        rep = op.bdf2_step(theta, omega, _dev(un), u, u_nm1=None if unm1 is None else _dev(unm1), force=_dev(f),
                           newton_rtol=1e-12, max_newton=30,
                           linear=dict(rtol=1e-11, restart=200, maxit=4000, precond="f32", cheb_degree=4))
        ug = u.cpu().numpy()
    err = relmax(ug, uo)
    print(f"dim={dim} first={first_step}: newton {rep['newton_iterations']} linear {rep['linear_iterations']} "
          f"res {rep['residual0']:.2e} -> {rep['residual']:.2e}; |u_gpu - u_oracle| / |u| = {err:.2e}")
    assert rep["rc"] == 0
    assert rep["residual"] <= 1e-12 * rep["residual0"]
    assert err < 1e-9


def test_bdf2_step_rejects_steady_mesh():
    mesh = small_mesh(2, 2, steady=1)
    with binding.Operator(mesh) as op:
        n = op.n_dofs
        u = torch.zeros(n, dtype=torch.float64, device="cuda")
        rep = op.bdf2_step(0.1, 1.0, u.clone(), u, check=False)
        assert rep["rc"] == binding.MNS_ERR_INVALID_ARG


def test_bdf2_steps_conserve_rotation_consistency():
    """Two consecutive steps with a rotating rotor (0.01 rad per step): the
    second step's history uses the first step's result; both converge and
    the GPU iterate matches the oracle sequence."""
    dt = 0.05
    mesh = small_mesh(2, 2, n_theta=8, steady=0, dt=dt, nu=0.02)
    un, unm1, f = _start_fields(mesh, 77)
    omega = 0.01 / dt
    thetas = [0.31, 0.32]
    ref = [unm1, un]
    for th in thetas:
        u_next, _ = _oracle_step(oracle_cfg(mesh, th, omega), ref[-1], ref[-2], f, ref[-1], dt)
        ref.append(u_next)
    with binding.Operator(mesh) as op:
        levels = [_dev(unm1), _dev(un)]
        for th in thetas:
            u = levels[-1].clone()
            rep = op.bdf2_step(th, omega, levels[-1], u, u_nm1=levels[-2], force=_dev(f), newton_rtol=1e-12,
                               max_newton=30, linear=dict(rtol=1e-11, restart=200, maxit=4000, cheb_degree=4))
            assert rep["rc"] == 0
            levels.append(u)
        for k in (2, 3):
            assert relmax(levels[k].cpu().numpy(), ref[k]) < 1e-9
    assert math.isfinite(float(np.abs(ref[-1]).max()))


def test_taylor_green_vortex_with_rotating_rotor():
    """The GPU time step on an exact solution (the Taylor-Green vortex, whose
    oracle run is pinned by its convergence rates): eight BDF2 + Newton steps
    with the rotor turning 0.05 rad per step, walls and the pinned pressure at
    the exact values of each new level.  The GPU sequence equals the oracle
    sequence and so has the same error against the exact field."""
    from tests import test_oracle_pins as pins

    nu, dt, omega, theta0, nsteps = 0.05, 0.05, 1.0, 0.2, 8
    mesh = dict(dim=2, degree=2, r_in=0.3, r_if=0.55, r_out=1.0, height=1.0, n_theta=32, n_r_rotor=4,
                n_r_stator=6, n_z=1, nu=nu, steady=0, dt=dt)

    def cfg(step):
        return oracle_cfg(mesh, theta0 + omega * step * dt, omega)

    cons = oracle.constrained(cfg(0))
    ref_err = pins._tgv_run(32, 4, 6, dt, nsteps * dt, omega, nu=nu, theta0=theta0)
    with binding.Operator(mesh) as op:
        levels = [_dev(pins._tgv_levels(cfg(-1), -dt, nu)), _dev(pins._tgv_levels(cfg(0), 0.0, nu))]
        for step in range(1, nsteps + 1):
            exact = pins._tgv_levels(cfg(step), step * dt, nu)
            guess = levels[-1].cpu().numpy()
            guess[cons] = exact[cons]
            u = _dev(guess)
            rep = op.bdf2_step(theta0 + omega * step * dt, omega, levels[-1], u, u_nm1=levels[-2],
                               newton_rtol=1e-12, max_newton=30,
                               linear=dict(rtol=1e-11, restart=200, maxit=4000, cheb_degree=4))
            assert rep["rc"] == 0, rep
            levels.append(u)
        err = pins._tgv_errors(levels[-1].cpu().numpy(), exact)
    print(f"Taylor-Green after {nsteps} steps: GPU velocity {err[0]:.4e} pressure {err[1]:.4e}; "
          f"oracle {ref_err[0]:.4e} {ref_err[1]:.4e}")
    assert abs(err[0] / ref_err[0] - 1.0) < 1e-6 and abs(err[1] / ref_err[1] - 1.0) < 1e-6
    assert err[0] < 2e-3 and err[1] < 3e-2


def _tgv3d(cfg, t, nu):
    """The Taylor-Green vortex of the 2D pin extended in z (u_z = 0, no z
    dependence): an exact solution of the 3D equations as well."""
    from tests import test_oracle_pins as pins

    kap = pins._TGV_KAPPA
    xyz = oracle.node_coords(cfg)
    x, y = xyz[:, 0], xyz[:, 1]
    f = math.exp(-2.0 * nu * kap * kap * t)
    out = np.zeros(4 * len(x))
    out[0::4] = np.sin(kap * x) * np.cos(kap * y) * f
    out[1::4] = -np.cos(kap * x) * np.sin(kap * y) * f
    out[3::4] = 0.25 * (np.cos(2 * kap * x) + np.cos(2 * kap * y)) * f * f
    return out


def _tgv3d_gpu(n_theta, n_r_rotor, n_r_stator, dt, t_end, nu=0.05, omega=1.0, theta0=0.2):
    mesh = dict(dim=3, degree=2, r_in=0.3, r_if=0.55, r_out=1.0, height=0.4, n_theta=n_theta, n_r_rotor=n_r_rotor,
                n_r_stator=n_r_stator, n_z=2, nu=nu, steady=0, dt=dt)

    def cfg(step):
        return oracle_cfg(mesh, theta0 + omega * step * dt, omega)

    cons = oracle.constrained(cfg(0))
    nsteps = int(round(t_end / dt))
    with binding.Operator(mesh) as op:
        levels = [_dev(_tgv3d(cfg(-1), -dt, nu)), _dev(_tgv3d(cfg(0), 0.0, nu))]
        for step in range(1, nsteps + 1):
            exact = _tgv3d(cfg(step), step * dt, nu)
            guess = levels[-1].cpu().numpy()
            guess[cons] = exact[cons]
            u = _dev(guess)
            rep = op.bdf2_step(theta0 + omega * step * dt, omega, levels[-1], u, u_nm1=levels[-2],
                               newton_rtol=1e-11, max_newton=30,
                               linear=dict(rtol=1e-10, restart=100, maxit=4000, cheb_degree=12))
            assert rep["rc"] == 0, rep
            levels.append(u)
        u = levels[-1].cpu().numpy()
    vel = np.arange(len(u)) % 4 < 3
    e = np.abs(u - exact)
    return e[vel].max() / np.abs(exact[vel]).max(), e[~vel].max() / np.abs(exact[~vel]).max()


def test_taylor_green_vortex_3d_converges():
    """3D time steps with the rotor turning on the z-extruded Taylor-Green
    vortex (walls, top and bottom at the exact values): the GPU solution
    converges to the exact field at the 2D pin's rates when h and dt halve
    (the z direction is resolved exactly), with errors of the 2D pin's size."""
    ev_c, ep_c = _tgv3d_gpu(16, 2, 3, 0.1, 0.4)
    ev_f, ep_f = _tgv3d_gpu(32, 4, 6, 0.05, 0.4)
    print(f"3D Taylor-Green: velocity {ev_c:.3e} -> {ev_f:.3e}, pressure {ep_c:.3e} -> {ep_f:.3e}")
    assert math.log2(ev_c / ev_f) > 3.0 and math.log2(ep_c / ep_f) > 2.0
    assert ev_f < 3e-3 and ep_f < 5e-2
