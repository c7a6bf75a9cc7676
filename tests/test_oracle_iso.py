"""Pins of the oracle's iso-parametric geometry (the Q_k mapping of the
paper's meshes, Sec. 2.1; the exact-circle mortar of Sec. 3.1 / Sec. 3.2 kept
on the interface): cells are the Q_k interpolants of their node positions,
which are the polar Gauss-Lobatto nodes moved by a smooth interior
perturbation that leaves the walls, the interface and the planes z = 0, H in
place.

Pins: affine fields are exact in the iso-parametric space (their physical
gradients are constant and their Laplacians vanish: the Jacobian and the
Hessian terms of the map); the enclosed area equals Green's theorem on the
interpolated boundary curves, computed here independently; interior moves
leave the total volume unchanged; the mortar measure stays 2 pi R H;
matrix-free = assembled, Newton consistency and the aligned reduction to the
conforming stabilized CG operator on a perturbed mesh; the discrete mass
balance is independent of the interior perturbation and converges at rate 4
(face interpolant against the exact arc); the manufactured solution converges
at the optimal Q2 rates on the perturbed mesh."""
import math

import numpy as np
import pytest

import oracle
from test_oracle_pins import _cfg, _merge_map, _solve_mms, _two_sided_field

PERT = 0.1  # mid nodes move by up to a tenth of a cell (a quarter makes a Q2 map singular)


def _iso(**kw):
    return _cfg(**dict(dict(iso=1, perturb=PERT), **kw))


@pytest.mark.parametrize("dim,k", [(2, 2), (2, 3), (3, 2), (3, 3)])
def test_affine_fields_are_exact(dim, k):
    """u = A x + b lies in the iso-parametric space (x itself is the Q_k
    interpolant of the nodes), so at any point of any perturbed cell the
    physical gradient of its interpolant is A and its Laplacian is 0.  A
    transposed Jacobian, a wrong inverse or a dropped Hessian-of-the-map term
    breaks this."""
    cfg = _iso(dim=dim, degree=k, n_theta=5, n_r_rotor=2, n_r_stator=2, n_z=2, theta_rot=0.7)
    X = oracle.node_coords(cfg)
    ncells = oracle.sizes(cfg)[2]
    g = np.random.default_rng(10 * dim + k)
    A = g.uniform(-1, 1, (3, 3))
    b = g.uniform(-1, 1, 3)
    U = X @ A.T + b  # nodal values of three affine fields
    for cell in g.choice(ncells, 6, replace=False):
        xi = g.uniform(0.05, 0.95, 3)
        phi, grad, lap, x = oracle.phys_basis(cfg, cell, xi[:dim])
        ids = _cell_nodes(cfg, cell)
        assert ids.size == phi.size == (k + 1) ** dim
        u = phi @ U[ids]
        gu = grad[:, :dim].T @ U[ids]  # gu[p, j] = d u_j / d x_p
        lu = lap @ U[ids]
        np.testing.assert_allclose(u, A @ x + b, rtol=0, atol=1e-13)
        np.testing.assert_allclose(gu.T, A[:, :dim], rtol=0, atol=1e-11)
        assert np.abs(lu).max() < 1e-9, lu


def _cell_nodes(cfg, cell):
    """Global node ids of a cell's local nodes in the oracle's local order
    (theta fastest, then r, then z), from the structured numbering."""
    dim, k = cfg["dim"], cfg["degree"]
    n = k + 1
    nt0 = cfg["n_theta"]
    nt1 = cfg.get("n_theta_stator") or nt0
    nr = (cfg["n_r_rotor"], cfg["n_r_stator"])
    nz = cfg["n_z"] if dim == 3 else 1
    nzn = k * nz + 1 if dim == 3 else 1
    ncell0 = nt0 * nr[0] * nz
    dom = 0 if cell < ncell0 else 1
    c = cell - (0 if dom == 0 else ncell0)
    nt = nt0 if dom == 0 else nt1
    ct, cr, cz = c % nt, (c // nt) % nr[dom], c // (nt * nr[dom])
    ntn = k * nt
    nrn = k * nr[dom] + 1
    off = 0 if dom == 0 else k * nt0 * (k * nr[0] + 1) * nzn
    ids = []
    for a2 in range(n if dim == 3 else 1):
        for a1 in range(n):
            for a0 in range(n):
                it = (k * ct + a0) % ntn
                ids.append(off + it + ntn * (k * cr + a1 + nrn * (k * cz + a2 if dim == 3 else 0)))
    return np.array(ids)


def _green_area(cfg):
    """Area between the Q_k interpolants of the outer and inner circles
    through their Gauss-Lobatto nodes, by Green's theorem: 1/2 of the
    integral of x dy - y dx along each interpolated arc (a polynomial in the
    face parameter, integrated exactly by a 20-point Gauss rule).  Written
    here from numpy's polynomial fitting, independent of the oracle."""
    k, nt = cfg["degree"], cfg["n_theta"]
    gll = oracle.rules(k + 1)[0]
    t, w = np.polynomial.legendre.leggauss(20)
    t, w = 0.5 * (t + 1), 0.5 * w
    total = 0.0
    for R, sign in ((cfg["r_out"], 1.0), (cfg["r_in"], -1.0)):
        for j in range(nt):
            th = (j + gll) * 2 * math.pi / nt
            px = np.polyfit(gll, R * np.cos(th), k)
            py = np.polyfit(gll, R * np.sin(th), k)
            x, y = np.polyval(px, t), np.polyval(py, t)
            dx, dy = np.polyval(np.polyder(px), t), np.polyval(np.polyder(py), t)
            total += sign * 0.5 * np.sum(w * (x * dy - y * dx))
    return total


@pytest.mark.parametrize("k", [2, 3])
def test_area_volume_and_interface_measure(k):
    """2D: the sum of the iso cells' areas equals Green's theorem on the
    interpolated boundary (exact quadrature of det J for Q_k cells); moving
    interior nodes changes no total area or volume (3D degree 2, where the
    cell quadrature of det J is exact too, as area x H); the mortar
    quadrature still integrates over the exact circle: sum JxW = 2 pi R H."""
    c2 = _iso(dim=2, degree=k, n_theta=7, n_r_rotor=2, n_r_stator=3, perturb=0.0)
    A0 = oracle.cell_info(c2)["V"].sum()
    assert abs(A0 - _green_area(c2)) < 1e-13 * A0
    Ap = oracle.cell_info(dict(c2, perturb=PERT))["V"].sum()
    assert abs(Ap - A0) < 1e-13 * A0
    exact = math.pi * (c2["r_out"] ** 2 - c2["r_in"] ** 2)
    assert 1e-6 < abs(A0 - exact) / exact < 1e-2  # the interpolated circles are not the circles
    if k == 2:
        c3 = _iso(dim=3, degree=2, n_theta=7, n_r_rotor=2, n_r_stator=3, n_z=3, height=1.3)
        V = oracle.cell_info(c3)["V"].sum()
        assert abs(V - A0 * 1.3) < 1e-13 * V
        _, _, jxw = oracle.segments(c3)
        assert abs(jxw.sum() - 2 * math.pi * c3["r_if"] * 1.3) < 1e-12


def test_node_perturbation_keeps_boundaries():
    """Walls, interface and the planes z = 0, H keep their nodes (radius and
    height unchanged); interior nodes move by a sizable part of a cell."""
    cfg = _iso(dim=3, n_theta=8, n_r_rotor=3, n_r_stator=3, n_z=3, theta_rot=0.4)
    X = oracle.node_coords(cfg)
    Xp = oracle.node_coords(dict(cfg, perturb=0.0))
    r, rp = np.hypot(X[:, 0], X[:, 1]), np.hypot(Xp[:, 0], Xp[:, 1])
    for R in (cfg["r_in"], cfg["r_if"], cfg["r_out"]):
        on = np.abs(rp - R) < 1e-12
        assert on.sum() > 0 and np.abs(r[on] - R).max() < 1e-12 and np.abs(X[on] - Xp[on]).max() < 1e-12
    for Z in (0.0, cfg["height"]):
        on = np.abs(Xp[:, 2] - Z) < 1e-12
        assert np.abs(X[on, 2] - Z).max() < 1e-12
    dr = (cfg["r_if"] - cfg["r_in"]) / 3
    assert np.abs(X - Xp).max() > 0.05 * dr
    # a perturbation that folds a cell is refused
    with pytest.raises(RuntimeError):
        oracle.node_coords(dict(cfg, perturb=0.8))


@pytest.mark.parametrize("dim", [2, 3])
def test_consistency_on_perturbed_mesh(dim):
    """Matrix-free = assembled (Alg. Alg-matrix for the faces) and Newton
    consistency (central differences of the residual with tau frozen,
    second order in eps) on a perturbed iso-parametric mesh, transient."""
    cfg = _iso(dim=dim, n_theta=4, n_r_rotor=1, n_r_stator=2, n_z=2, theta_rot=0.9, steady=0, dt=0.05)
    n = oracle.n_dofs(cfg)
    g = np.random.default_rng(21 + dim)
    u, x, hist, f = (g.uniform(-1, 1, n) for _ in range(4))
    cons = oracle.constrained(cfg)
    x[cons] = 0
    y = oracle.apply_jacobian(cfg, u, x, hist=hist, force=f)
    A = oracle.assemble(cfg, u, hist, f)
    assert np.abs(A @ x - y).max() <= 1e-13 * np.abs(y).max()
    errs = []
    for eps in (1e-2, 1e-3):  # the BDF2 mass term dominates y: larger steps keep the O(eps^2) part visible
        fd = (oracle.residual(cfg, u + eps * x, hist, f, tau_state=u) -
              oracle.residual(cfg, u - eps * x, hist, f, tau_state=u)) / (2 * eps)
        errs.append(np.abs(fd - y)[~cons].max() / np.abs(y).max())
    assert errs[1] < 3e-7 and errs[0] / errs[1] > 60, errs


@pytest.mark.parametrize("dim", [2, 3])
def test_aligned_mortar_reduces_to_conforming_cg_on_perturbed_mesh(dim):
    """At an aligned angle the two sides' interface faces are the same
    interpolated curve through the same nodes, so E^T J_mortar E equals the
    stabilized CG operator of the merged conforming iso-parametric mesh with
    the same perturbed nodes."""
    cfg = _iso(dim=dim, theta_rot=0.0)
    E = _merge_map(cfg)
    g = np.random.default_rng(19)
    ug = g.uniform(-1, 1, E.shape[1])
    Jm = oracle.assemble(cfg, E @ ug)
    cg = dict(cfg, merged=1)
    Jg = oracle.assemble(cg, ug)
    free = ~oracle.constrained(cg)
    D = (E.T @ Jm @ E - Jg).toarray()[np.ix_(free, free)]
    assert np.abs(D).max() < 1e-13 * abs(Jg).max()


@pytest.mark.parametrize("dim", [2, 3])
def test_mass_balance_on_iso_mesh(dim):
    """Sum of the pressure rows of J x (test function q = 1): the volume part
    integrates div(du) exactly on every iso cell (det J times the physical
    divergence is a polynomial of the quadrature's exact degree), so moving
    interior nodes does not change the sum at all; what remains is the
    interface, whose mortar terms live on the exact circle while the cells'
    faces are its Q2 interpolants: that defect falls at rate 4."""
    errs = []
    for nt in (8, 16, 32):
        c = max(1, nt // 8)
        cfg = _iso(dim=dim, n_theta=nt, n_r_rotor=c, n_r_stator=c, n_z=c, pin_pressure=0)
        n = oracle.n_dofs(cfg)
        u = np.random.default_rng(3).uniform(-1, 1, n)
        pr = np.arange(n) % (dim + 1) == dim
        sums, mags = [], []
        for pert in (PERT, 0.0):
            cp = dict(cfg, perturb=pert)
            y = oracle.apply_jacobian(cp, u, _two_sided_field(cp, 4))[pr]
            sums.append(y.sum())
            mags.append(np.abs(y).sum())
        # equal up to the rounding of the sum (the rows themselves change)
        assert abs(sums[0] - sums[1]) < 1e-13 * mags[1], (sums, mags)
        errs.append(abs(sums[0]))
    r1, r2 = math.log2(errs[0] / errs[1]), math.log2(errs[1] / errs[2])
    assert r1 > 3.5 and r2 > 3.5, errs


@pytest.mark.slow
def test_mms_convergence_q2_perturbed_iso():
    """Whole discretization on the perturbed iso-parametric mesh (2D Q2,
    nu = 1, rotor at 0.05 rad): the manufactured solution converges at the
    optimal O(h^3) velocity and O(h^2) pressure rates."""
    errs = []
    for nt, nr in ((16, 2), (32, 4), (64, 8)):
        cfg = oracle.params(dim=2, degree=2, n_theta=nt, n_r_rotor=nr, n_r_stator=nr, nu=1.0, omega=0.0,
                            theta_rot=0.05, mms=1, nthreads=0, iso=1, perturb=PERT)
        errs.append(oracle.mms_errors(cfg, _solve_mms(cfg)))
    for a, b in zip(errs, errs[1:]):
        ru, rp = math.log2(a[0] / b[0]), math.log2(a[1] / b[1])
        assert ru > 3.0 - 0.25 and rp > 2.0 - 0.25, (ru, rp, errs)
