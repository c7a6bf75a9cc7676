"""Pins of the FP64 oracle against facts the paper and the mathematics fix.

Each test names the part of the oracle it pins and the kind of pin (closed form,
library routine, brute force, exact invariant, convergence order).  None of them
re-types the oracle's formula; together they are chosen so that a dropped term,
a wrong sign or index, or a transposed operand in any part fails at least one
(tests/test_oracle_mutants.py plants such mistakes and checks exactly that).
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import oracle


def _cfg(**kw):
    base = dict(dim=2, degree=2, r_in=0.25, r_if=0.5, r_out=1.0, height=1.0, n_theta=6, n_r_rotor=1,
                n_r_stator=2, n_z=2, nu=0.07, omega=0.6, theta_rot=0.21)
    base.update(kw)
    return oracle.params(**base)


def _blocks(cfg):
    n = oracle.n_dofs(cfg)
    comp = np.arange(n) % (cfg["dim"] + 1)
    free = ~oracle.constrained(cfg)
    return (comp < cfg["dim"]) & free, (comp == cfg["dim"]) & free


# ---------------------------------------------------------------- 1D rules --

@pytest.mark.parametrize("n", [2, 3, 4, 5, 6, 7])
def test_gauss_rule_matches_library_and_exactness(n):
    """Gauss-Legendre on [0,1]: equals numpy's leggauss mapped to [0,1] and
    integrates x^p exactly for p <= 2n-1 (library routine + closed form)."""
    gll, gx, gw = oracle.rules(n)
    t, w = np.polynomial.legendre.leggauss(n)
    np.testing.assert_allclose(gx, 0.5 * (t + 1), rtol=0, atol=1e-15)
    np.testing.assert_allclose(gw, 0.5 * w, rtol=0, atol=1e-15)
    for p in range(2 * n):
        assert abs(np.dot(gw, gx ** p) - 1.0 / (p + 1)) < 1e-14


@pytest.mark.parametrize("n", [2, 3, 4, 5, 6, 7])
def test_lobatto_nodes(n):
    """GLL nodes: 0, 1 and the roots of P'_{n-1} (numpy's Legendre routines);
    closed forms for n = 3, 4, 5."""
    gll, _, _ = oracle.rules(n)
    assert gll[0] == 0.0 and gll[-1] == 1.0
    if n > 2:
        roots = np.sort(np.polynomial.legendre.Legendre.basis(n - 1).deriv().roots().real)
        np.testing.assert_allclose(gll[1:-1], 0.5 * (roots + 1), atol=1e-14)
    closed = {3: [0, 0.5, 1], 4: [0, (1 - 1 / math.sqrt(5)) / 2, (1 + 1 / math.sqrt(5)) / 2, 1],
              5: [0, (1 - math.sqrt(3 / 7)) / 2, 0.5, (1 + math.sqrt(3 / 7)) / 2, 1]}
    if n in closed:
        np.testing.assert_allclose(gll, closed[n], atol=1e-15)


@pytest.mark.parametrize("n", [3, 4, 5, 6])
def test_lagrange_basis(n):
    """Partition of unity, cardinality at the nodes, and exact interpolation of
    every polynomial of degree <= n-1 with its first and second derivatives."""
    gll, _, _ = oracle.rules(n)
    for t in [0.0, 0.13, 0.5, 0.77, 1.0] + list(gll):
        L, dL, d2L = oracle.lagrange(gll, t)
        assert abs(L.sum() - 1) < 1e-13 and abs(dL.sum()) < 1e-11 and abs(d2L.sum()) < 1e-9
        for p in range(n):
            f = gll ** p
            assert abs(L @ f - t ** p) < 1e-13
            assert abs(dL @ f - (p * t ** (p - 1) if p >= 1 else 0)) < 1e-11
            assert abs(d2L @ f - (p * (p - 1) * t ** (p - 2) if p >= 2 else 0)) < 1e-9
    for j, xj in enumerate(gll):
        L, _, _ = oracle.lagrange(gll, xj)
        np.testing.assert_allclose(L, np.eye(n)[j], atol=1e-14)


# ---------------------------------------------------------------- geometry --

@pytest.mark.parametrize("dim", [2, 3])
def test_cell_measures_sum_to_annulus(dim):
    """Sum of cell areas (volumes) = pi (r_out^2 - r_in^2) [H]; per cell the
    polar closed form (r1^2 - r0^2) dtheta / 2 [dz]."""
    cfg = _cfg(dim=dim, n_theta=7, n_r_rotor=2, n_r_stator=3, n_z=3, height=1.3)
    info = oracle.cell_info(cfg)
    H = cfg["height"] if dim == 3 else 1.0
    total = math.pi * (cfg["r_out"] ** 2 - cfg["r_in"] ** 2) * H
    assert abs(info["V"].sum() - total) < 1e-13 * total
    dth = 2 * math.pi / cfg["n_theta"]
    dz = H / cfg["n_z"] if dim == 3 else 1.0
    dr = (cfg["r_if"] - cfg["r_in"]) / 2
    V0 = 0.5 * ((cfg["r_in"] + dr) ** 2 - cfg["r_in"] ** 2) * dth * dz
    assert abs(info["V"][0] - V0) < 1e-15
    h0 = 2 * math.sqrt(V0 / math.pi) if dim == 2 else (6 * V0 / math.pi) ** (1 / 3)
    assert abs(info["h"][0] - h0) < 1e-15


@pytest.mark.parametrize("dim", [2, 3])
def test_penalty_closed_form(dim):
    """Eq. EqPenalty on one rotor and one stator interface cell, written with
    the polar face measures: mortar face R dtheta [dz]; other faces the inner
    (outer) arc, two radial edges and, in 3D, two annular sectors."""
    cfg = _cfg(dim=dim, degree=3, n_theta=9, n_r_rotor=2, n_r_stator=3, n_z=4, penalty_F=2.5)
    info = oracle.cell_info(cfg)
    k, F, R = 3, 2.5, cfg["r_if"]
    dth = 2 * math.pi / 9
    dz = 1.0 / 4 if dim == 3 else 1.0

    def tau(r0, r1, mortar_r, other_r):
        V = 0.5 * (r1 ** 2 - r0 ** 2) * dth * dz
        A_m = mortar_r * dth * dz
        A_o = other_r * dth * dz + 2 * (r1 - r0) * dz
        if dim == 3:
            A_o += 2 * 0.5 * (r1 ** 2 - r0 ** 2) * dth
        return F * (k + 1) ** 2 * (0.5 * A_o + A_m) / V

    dr_r = (R - cfg["r_in"]) / 2
    dr_s = (cfg["r_out"] - R) / 3
    t_rot = tau(R - dr_r, R, R, R - dr_r)
    t_sta = tau(R, R + dr_s, R, R + dr_s)
    np.testing.assert_allclose(info["tau_side"], [t_rot, t_sta], rtol=1e-14)
    info1 = oracle.cell_info(dict(cfg, penalty_rule=1))
    np.testing.assert_allclose(info1["tau_side"], [max(t_rot, t_sta)] * 2, rtol=1e-14)


@pytest.mark.parametrize("dim,k", [(2, 2), (2, 3), (3, 2), (3, 3)])
def test_physical_derivatives_of_polar_polynomials(dim, k):
    """The generic chain rule (with mapping second derivatives) applied to
    fields exactly representable on a polar cell: f = r^2 theta (+ z^2) has
    grad f = 2 r theta e_r + r e_theta (+ 2 z e_z) and
    lap f = 4 theta (+ 2) in the plane (closed form)."""
    cfg = _cfg(dim=dim, degree=k, theta_rot=0.37)
    n = k + 1
    gll, _, _ = oracle.rules(n)
    cell = 3  # a rotor cell (rotated by theta_rot)
    dth = 2 * math.pi / cfg["n_theta"]
    r0 = cfg["r_in"]
    dr = (cfg["r_if"] - cfg["r_in"]) / cfg["n_r_rotor"]
    th0 = cfg["theta_rot"] + cell * dth
    dz = cfg["height"] / cfg["n_z"]
    # nodal values from the node positions of the polar map
    nd = n ** dim
    idx = np.array(np.unravel_index(np.arange(nd), (n,) * dim, order="F")).T
    th = th0 + dth * gll[idx[:, 0]]
    r = r0 + dr * gll[idx[:, 1]]
    f = r ** 2 * th
    if dim == 3:
        f = f + (dz * gll[idx[:, 2]]) ** 2
    for xi in [(0.2, 0.7, 0.4), (0.9, 0.1, 0.55)]:
        phi, grad, lap, x = oracle.phys_basis(cfg, cell, xi[:dim])
        rr = math.hypot(x[0], x[1])
        tt = th0 + dth * xi[0]
        er = np.array([math.cos(tt), math.sin(tt), 0])
        et = np.array([-math.sin(tt), math.cos(tt), 0])
        g_ex = 2 * rr * tt * er + rr * et
        lap_ex = 4 * tt
        if dim == 3:
            g_ex = g_ex + np.array([0, 0, 2 * x[2]])
            lap_ex += 2
        assert abs(phi @ f - (rr ** 2 * tt + (x[2] ** 2 if dim == 3 else 0))) < 1e-13
        np.testing.assert_allclose(grad.T @ f, g_ex, atol=1e-11)
        assert abs(lap @ f - lap_ex) < 1e-8


# ------------------------------------------------------------------ mortar --

@pytest.mark.parametrize("dim", [2, 3])
def test_mortar_segments(dim):
    """Sec. 3.2: one segment per face when aligned, two otherwise; the mapped
    quadrature integrates the interface exactly at every angle: sum JxW =
    2 pi R [H], and per stator face R dtheta [dz]; each segment lies inside
    both paired faces."""
    nt, nz = 8, 3
    dth = 2 * math.pi / nt
    for theta in [0.0, 0.3 * dth, dth, 2.9, 5 * dth + 1e-3, 2 * math.pi - 1e-3, -0.7]:
        cfg = _cfg(dim=dim, n_theta=nt, n_z=nz, theta_rot=theta)
        ids, lohi, jxw = oracle.segments(cfg)
        layers = nz if dim == 3 else 1
        phi = (theta % dth)
        aligned = min(phi, dth - phi) < 1e-12 * dth
        assert len(ids) == (1 if aligned else 2) * nt * layers
        H = cfg["height"] if dim == 3 else 1.0
        assert abs(jxw.sum() - 2 * math.pi * cfg["r_if"] * H) < 1e-12
        n = cfg["degree"] + 1
        per = jxw.reshape(len(ids), -1).sum(axis=1)
        face_sum = np.zeros((layers, nt))
        np.add.at(face_sum, (ids[:, 0], ids[:, 2]), per)
        np.testing.assert_allclose(face_sum, cfg["r_if"] * dth * H / layers, rtol=1e-13)
        for (cz, ir, js), (lo, hi) in zip(ids, lohi):
            assert js * dth - 1e-12 <= lo < hi <= (js + 1) * dth + 1e-12
            rot_lo = (theta + ir * dth - lo) % (2 * math.pi)
            assert rot_lo < 1e-9 or rot_lo > 2 * math.pi - dth - 1e-9


# ------------------------------ unequal interface counts (Sec. 3.1, Sec. 5) --
# The rotor and stator rings may hold different cell counts; a face then meets
# more than two faces of the other side and every intersection is a mortar
# segment with its own mapped quadrature.

UNEQUAL = [(6, 8), (8, 12), (12, 8), (5, 7)]


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("ntr,nts", UNEQUAL)
def test_mortar_segments_unequal_counts(dim, ntr, nts):
    """Segments are the intersections of rotor and stator faces: the breakpoints
    of both rings (the union minus coincidences) split each layer into
    segments; the mapped quadrature integrates the interface exactly at every
    angle (sum JxW = 2 pi R [H]) and each face of either side exactly
    (R dtheta_side [dz]); every segment lies inside both of its faces."""
    nz = 3
    dr_, ds_ = 2 * math.pi / ntr, 2 * math.pi / nts
    for theta in [0.0, 0.3 * dr_, 2.9, dr_ * 3 + 1e-3, -0.7]:
        cfg = _cfg(dim=dim, n_theta=ntr, n_theta_stator=nts, n_z=nz, theta_rot=theta)
        ids, lohi, jxw = oracle.segments(cfg)
        layers = nz if dim == 3 else 1
        H = cfg["height"] if dim == 3 else 1.0
        # breakpoints on the circle, in [0, 2 pi)
        pts = sorted({round((j * ds_) % (2 * math.pi), 10) for j in range(nts)} |
                     {round((theta + i * dr_) % (2 * math.pi), 10) for i in range(ntr)})
        merged = [p for i, p in enumerate(pts) if i == 0 or p - pts[i - 1] > 1e-9]
        if len(merged) > 1 and merged[-1] - merged[0] > 2 * math.pi - 1e-9:
            merged.pop()
        assert len(ids) == len(merged) * layers
        assert abs(jxw.sum() - 2 * math.pi * cfg["r_if"] * H) < 1e-12
        per = jxw.reshape(len(ids), -1).sum(axis=1)
        st, rt = np.zeros((layers, nts)), np.zeros((layers, ntr))
        np.add.at(st, (ids[:, 0], ids[:, 2]), per)
        np.add.at(rt, (ids[:, 0], ids[:, 1]), per)
        np.testing.assert_allclose(st, cfg["r_if"] * ds_ * H / layers, rtol=1e-13)
        np.testing.assert_allclose(rt, cfg["r_if"] * dr_ * H / layers, rtol=1e-13)
        for (cz, ir, js), (lo, hi) in zip(ids, lohi):
            assert js * ds_ - 1e-12 <= lo < hi <= (js + 1) * ds_ + 1e-12
            off = (lo - theta - ir * dr_ + math.pi) % (2 * math.pi) - math.pi  # signed, in [-pi, pi)
            assert -1e-9 <= off and off + (hi - lo) <= dr_ + 1e-9


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("ntr,nts", [(6, 8), (8, 6)])
def test_unequal_counts_structure(dim, ntr, nts):
    """With unequal interface counts: matrix-free = assembled (Alg. Alg-matrix),
    Alg. Alg-diagonal = assembled diagonal, Newton consistency with the
    residual (O(eps^2)), B = -C^T with stabilization off, and SIPG symmetry
    with equal penalties."""
    cfg = _cfg(dim=dim, n_theta=ntr, n_theta_stator=nts, n_z=2, theta_rot=0.61, steady=0, dt=0.05)
    n = oracle.n_dofs(cfg)
    g = np.random.default_rng(31)
    u, x = g.uniform(-1, 1, n), g.uniform(-1, 1, n)
    hist = g.uniform(-1, 1, n)
    A = oracle.assemble(cfg, u, hist)
    y = oracle.apply_jacobian(cfg, u, x, hist=hist)
    assert np.abs(A @ x - y).max() <= 1e-13 * np.abs(y).max()
    np.testing.assert_allclose(oracle.diagonal(cfg, u, hist), A.diagonal(), rtol=1e-12, atol=1e-14)
    cons = oracle.constrained(cfg)
    xm = x.copy()
    xm[cons] = 0
    ym = oracle.apply_jacobian(cfg, u, xm, hist=hist)
    errs = []
    for eps in (1e-3, 1e-4):
        fd = (oracle.residual(cfg, u + eps * xm, hist, tau_state=u) -
              oracle.residual(cfg, u - eps * xm, hist, tau_state=u)) / (2 * eps)
        errs.append(np.abs(fd - ym)[~cons].max() / np.abs(ym).max())
    assert errs[1] < 3e-8 and errs[0] / errs[1] > 60
    c0 = dict(cfg, stabilization=0, pin_pressure=0, steady=1)
    A0 = oracle.assemble(c0, np.zeros(n)).toarray()
    vel, pr = _blocks(c0)
    B, C = A0[np.ix_(vel, pr)], A0[np.ix_(pr, vel)]
    assert np.abs(B).max() > 1e-2 and np.abs(B + C.T).max() < 1e-14
    c1 = dict(cfg, stabilization=0, omega=0.0, penalty_rule=1, steady=1)
    Avv = oracle.assemble(c1, np.zeros(n)).toarray()[np.ix_(vel, vel)]
    assert np.abs(Avv - Avv.T).max() < 1e-14 * np.abs(Avv).max()


@pytest.mark.parametrize("dim", [2, 3])
def test_discrete_mass_conservation_unequal_counts(dim):
    """The mass balance of the pressure rows (Eq. EqMortarMass) with stator
    rings of 3/2 the rotor's cell count: quadrature-level zero, decaying
    under refinement."""
    errs, scale = [], []
    for nt in (8, 16, 32):
        c = max(1, nt // 8)
        cfg = _cfg(dim=dim, n_theta=nt, n_theta_stator=3 * nt // 2, n_r_rotor=c, n_r_stator=c, n_z=c,
                   pin_pressure=0)
        n = oracle.n_dofs(cfg)
        u = np.random.default_rng(3).uniform(-1, 1, n)
        yv = oracle.apply_jacobian(cfg, u, _two_sided_field(cfg, 4))
        pr = np.arange(n) % (dim + 1) == dim
        errs.append(abs(yv[pr].sum()))
        scale.append(np.abs(yv[pr]).max())
    r1, r2 = np.log2(errs[0] / errs[1]), np.log2(errs[1] / errs[2])
    assert r1 > 5.0 and r2 > 5.0, errs  # 7.6 and 5.9 in 2D: the finest level nears round-off
    assert errs[-1] < 1e-8 * scale[-1], (errs, scale)


# ----------------------------------- closed forms on one interior cell (2D) --
# Rows of J at the interior node of one cell couple only that cell's nodes, so
# special increments and states reduce them to integrals of the basis over the
# cell, evaluated here with the cell's Gauss rule (pinned above) and the
# closed-form polar Jacobian r dr dtheta.

def _interior_cell_setup(**kw):
    cfg = _cfg(dim=2, degree=2, n_theta=6, n_r_rotor=3, n_r_stator=2, omega=0.0, theta_rot=0.37, **kw)
    k, nt = 2, cfg["n_theta"]
    ct, cr = 2, 1                                     # rotor cell away from every wall and the interface
    cell = ct + nt * cr
    node = (k * ct + 1) + (k * nt) * (k * cr + 1)     # its interior node (theta fastest, rotor first)
    n = k + 1
    _, gx, gw = oracle.rules(n)
    dr = (cfg["r_if"] - cfg["r_in"]) / cfg["n_r_rotor"]
    dth = 2 * math.pi / nt
    pts = []
    for j in range(n):
        for i in range(n):
            phi, grad, _, x = oracle.phys_basis(cfg, cell, (gx[i], gx[j]))
            r = math.hypot(x[0], x[1])
            pts.append((phi, grad, x, r, gw[i] * gw[j] * r * dr * dth))
    phi_c, _, _, xc = oracle.phys_basis(cfg, cell, (0.5, 0.5))
    assert np.abs(oracle.node_coords(cfg)[node] - xc).max() < 1e-14   # the node is the cell centre
    a = 4                                                              # its local index (1, 1)
    assert abs(phi_c[a] - 1.0) < 1e-14
    r0 = cfg["r_in"] + cr * dr
    A = 0.5 * ((r0 + dr) ** 2 - r0 ** 2) * dth
    return cfg, cell, node, a, pts, A


@pytest.mark.parametrize("U,steady", [(0.0, 1), (0.7, 1), (0.7, 0)])
def test_tau_closed_form(U, steady):
    """Eq. Eq-stab-param through the PSPG block: for a uniform state u = (U, 0),
    p = 0, omega = 0 the pressure-pressure entry at a cell-interior node is
    tau (grad psi, grad psi) with tau = (c^2 + (2U/h)^2 + 9 (4 nu / h^2)^2)^(-1/2),
    c = 1/dt (0 when steady), h = 2 sqrt(A / pi)."""
    cfg, cell, node, a, pts, A = _interior_cell_setup(steady=steady, dt=0.05, nu=0.03)
    n = oracle.n_dofs(cfg)
    state = np.zeros(n)
    state[0::3] = U
    i = 3 * node + 2
    x = np.zeros(n)
    x[i] = 1.0
    Jii = oracle.apply_jacobian(cfg, state, x)[i]
    K = sum(w * grad[a] @ grad[a] for _, grad, _, _, w in pts)
    h = 2 * math.sqrt(A / math.pi)
    c = 0.0 if steady else 1.0 / 0.05
    tau = (c * c + (2 * U / h) ** 2 + 9 * (4 * 0.03 / h ** 2) ** 2) ** -0.5
    assert abs(Jii - tau * K) < 1e-13 * tau * K


@pytest.mark.parametrize("steady", [1, 0])
def test_mass_and_viscous_coefficients(steady):
    """Eq. Eq-discrete-1 at u = 0, omega = 0 (a = 0, R = 0, so no SUPG term):
    the velocity diagonal entry at a cell-interior node is
    c_t (psi, psi) + nu (grad psi, grad psi), c_t = 3 / (2 dt) for BDF2."""
    cfg, cell, node, a, pts, _ = _interior_cell_setup(steady=steady, dt=0.05, nu=0.03)
    n = oracle.n_dofs(cfg)
    i = 3 * node
    x = np.zeros(n)
    x[i] = 1.0
    y = oracle.apply_jacobian(cfg, np.zeros(n), x)
    Mii = sum(w * phi[a] ** 2 for phi, _, _, _, w in pts)
    Kii = sum(w * grad[a] @ grad[a] for _, grad, _, _, w in pts)
    ct = 0.0 if steady else 1.5 / 0.05
    assert abs(y[i] - (ct * Mii + 0.03 * Kii)) < 1e-13 * abs(y[i])
    assert abs(y[i + 1]) < 1e-15 * abs(y[i])


def test_ale_convection_of_rigid_rotation():
    """Sec. 3.1 mesh velocity u_ALE = omega e_z x x in the convective term: with
    u = 0 the advecting velocity is a = -u_ALE, and the increment
    du_x = theta - theta_c (exact on the cell) has grad du_x = e_theta / r, so
    the row of the cell-interior node is -omega (psi, 1) + nu (grad psi, e_theta / r)."""
    omega, nu = 0.8, 0.03
    cfg, cell, node, a, pts, _ = _interior_cell_setup(nu=nu, stabilization=0)
    cfg = dict(cfg, omega=omega)
    n = oracle.n_dofs(cfg)
    xyz = oracle.node_coords(cfg)
    xc = xyz[node]
    k, nt = 2, cfg["n_theta"]
    x = np.zeros(n)
    ct, cr = 2, 1
    for b in range(k + 1):
        for a0 in range(k + 1):
            nd = (k * ct + a0) + (k * nt) * (k * cr + b)
            p = xyz[nd]
            x[3 * nd] = math.atan2(xc[0] * p[1] - xc[1] * p[0], xc[0] * p[0] + xc[1] * p[1])
    y = oracle.apply_jacobian(cfg, np.zeros(n), x)
    exp = 0.0
    for phi, grad, xq, r, w in pts:
        et = np.array([-xq[1], xq[0], 0.0]) / r
        exp += w * (-omega * phi[a] + nu * grad[a] @ et / r)
    assert abs(exp) > 1e-3
    assert abs(y[3 * node] - exp) < 1e-12 * abs(exp)


def test_interface_penalty_closed_form():
    """Eq. EqPenalty in the face term: only the penalty depends on F, so for the
    velocity DoF of a rotor interface node inside one face, J_ii(F=3) - J_ii(F=1)
    = nu (tau_rot(3) - tau_rot(1)) R dtheta * integral of L_1^2 over the face
    (Gauss rule exact for this degree; tau_rot from its own closed-form pin)."""
    nt, k, nu = 6, 2, 0.07
    dth = 2 * math.pi / nt
    cfg = _cfg(dim=2, degree=k, n_theta=nt, n_r_rotor=2, n_r_stator=2, nu=nu, theta_rot=2 * dth, omega=0.0)
    n = oracle.n_dofs(cfg)
    node = (k * 1 + 1) + (k * nt) * (k * cfg["n_r_rotor"])   # rotor cell 1, face-interior node on r = R
    i = 3 * node
    x = np.zeros(n)
    x[i] = 1.0
    J = {F: oracle.apply_jacobian(dict(cfg, penalty_F=F), np.zeros(n), x)[i] for F in (1.0, 3.0)}
    tau = {F: oracle.cell_info(dict(cfg, penalty_F=F))["tau_side"][0] for F in (1.0, 3.0)}
    gll, gx, gw = oracle.rules(k + 1)
    face = cfg["r_if"] * dth * sum(w * oracle.lagrange(gll, t)[0][1] ** 2 for t, w in zip(gx, gw))
    exp = nu * (tau[3.0] - tau[1.0]) * face
    assert abs((J[3.0] - J[1.0]) - exp) < 1e-12 * exp


# --------------------------------------------- operator: brute force checks --

@pytest.mark.parametrize("dim", [2, 3])
def test_matrix_free_equals_assembled(dim):
    """Gather, scatter, constraints and mortar pairing: oracle vmult equals the
    COO matrix assembled column by column (Alg. Alg-matrix for the faces)."""
    cfg = _cfg(dim=dim, n_theta=4, n_r_rotor=1, n_r_stator=1, n_z=2, theta_rot=0.5)
    n = oracle.n_dofs(cfg)
    g = np.random.default_rng(5)
    state, x = g.uniform(-1, 1, n), g.uniform(-1, 1, n)
    A = oracle.assemble(cfg, state)
    y = oracle.apply_jacobian(cfg, state, x)
    assert np.abs(A @ x - y).max() <= 1e-13 * np.abs(y).max()


@pytest.mark.parametrize("dim", [2, 3])
def test_diagonal_and_rows(dim):
    """Alg. Alg-diagonal equals the assembled diagonal; sampled rows equal the
    full product."""
    cfg = _cfg(dim=dim, n_theta=4, n_r_rotor=1, n_r_stator=1, n_z=2, theta_rot=2.0)
    n = oracle.n_dofs(cfg)
    g = np.random.default_rng(6)
    state, x = g.uniform(-1, 1, n), g.uniform(-1, 1, n)
    A = oracle.assemble(cfg, state)
    np.testing.assert_allclose(oracle.diagonal(cfg, state), A.diagonal(), rtol=1e-12, atol=1e-14)
    rows = g.choice(n, 40, replace=False)
    y = oracle.apply_jacobian(cfg, state, x)
    np.testing.assert_allclose(oracle.apply_jacobian_rows(cfg, state, x, rows), y[rows], rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("dim,steady", [(2, 1), (2, 0), (3, 1), (3, 0)])
def test_jacobian_is_derivative_of_residual(dim, steady):
    """Newton consistency (Eq. Eq-Newton-method): J x = [R(u+eps x) - R(u-eps x)]
    / (2 eps) with tau frozen at u; second-order convergence in eps.  Covers
    the SUPG weight derivative, B-hat and the BDF2 terms."""
    cfg = _cfg(dim=dim, steady=steady, dt=0.05, theta_rot=0.9)
    n = oracle.n_dofs(cfg)
    g = np.random.default_rng(7)
    u, x = g.uniform(-1, 1, n), g.uniform(-1, 1, n)
    hist, f = g.uniform(-1, 1, n), g.uniform(-1, 1, n)
    cons = oracle.constrained(cfg)
    x[cons] = 0
    y = oracle.apply_jacobian(cfg, u, x, hist=hist, force=f)
    errs = []
    for eps in (1e-3, 1e-4):
        fd = (oracle.residual(cfg, u + eps * x, hist, f, tau_state=u) -
              oracle.residual(cfg, u - eps * x, hist, f, tau_state=u)) / (2 * eps)
        errs.append(np.abs(fd - y)[~cons].max() / np.abs(y).max())
    assert errs[1] < 3e-8
    assert errs[0] / errs[1] > 60  # O(eps^2)


@pytest.mark.parametrize("dim,steady", [(2, 1), (2, 0), (3, 1)])
def test_picard_jacobian_applied_to_state_is_residual(dim, steady):
    """Picard (Oseen) option: every term of the residual is linear in u once the
    convection velocity u - u_ALE and the SUPG weight are frozen, so with no
    history and no forcing J_picard(u) u = R(u) (tau frozen at u).  The Newton
    Jacobian differs by the reaction term (du . grad) u and the SUPG weight
    derivative, which are nonzero here."""
    cfg = _cfg(dim=dim, steady=steady, dt=0.05, theta_rot=0.9)
    n = oracle.n_dofs(cfg)
    u = np.random.default_rng(11).uniform(-1, 1, n)
    u[oracle.constrained(cfg)] = 0
    r = oracle.residual(cfg, u)
    yp = oracle.apply_jacobian(dict(cfg, picard=1), u, u)
    yn = oracle.apply_jacobian(cfg, u, u)
    assert np.abs(r).max() > 1e-2
    assert np.abs(yp - r).max() < 1e-13 * np.abs(r).max()
    assert np.abs(yn - r).max() > 1e-2 * np.abs(r).max()
    # at u = 0 (convection by -u_ALE only) both linearizations coincide
    z = np.zeros(n)
    assert np.array_equal(oracle.apply_jacobian(dict(cfg, picard=1), z, u), oracle.apply_jacobian(cfg, z, u))


# ------------------------------------------------------ exact invariants --

@pytest.mark.parametrize("dim", [2, 3])
def test_galerkin_saddle_structure(dim):
    """Eqs. Eq-discrete-2/-3 with the per-side jump and normal: with
    stabilization off, B = -C^T exactly, mortar pressure flux and strong-DG
    mass term included."""
    cfg = _cfg(dim=dim, stabilization=0, pin_pressure=0)
    A = oracle.assemble(cfg, np.zeros(oracle.n_dofs(cfg))).toarray()
    vel, pr = _blocks(cfg)
    B, C = A[np.ix_(vel, pr)], A[np.ix_(pr, vel)]
    assert np.abs(B).max() > 1e-2
    assert np.abs(B + C.T).max() < 1e-14


@pytest.mark.parametrize("dim", [2, 3])
def test_sipg_symmetry(dim):
    """SIPG viscous block (Eq. EqMortarDiff) is symmetric when both sides use the
    same penalty (rule 1), and not with the per-cell penalties (rule 0) since
    tau_k differs between the sides here."""
    cfg = _cfg(dim=dim, stabilization=0, omega=0.0)
    A = oracle.assemble(dict(cfg, penalty_rule=1), np.zeros(oracle.n_dofs(cfg))).toarray()
    vel, _ = _blocks(cfg)
    Avv = A[np.ix_(vel, vel)]
    assert np.abs(Avv - Avv.T).max() < 1e-14 * np.abs(Avv).max()
    A0 = oracle.assemble(cfg, np.zeros(oracle.n_dofs(cfg))).toarray()[np.ix_(vel, vel)]
    assert np.abs(A0 - A0.T).max() > 1e-3


@pytest.mark.parametrize("dim", [2, 3])
def test_supg_pspg_adjoint_identity(dim):
    """With u = 0, nu = 0 and steady flow the SUPG part of B-hat equals the
    transpose of the PSPG part of C-hat: both are (tau (a.grad) phi_i, grad
    psi_j), reached through the test-side weight and the trial-side R'; the
    PSPG block D-hat is symmetric."""
    cfg = _cfg(dim=dim, nu=0.0, omega=0.9, pin_pressure=0)
    z = np.zeros(oracle.n_dofs(cfg))
    As = oracle.assemble(cfg, z).toarray()
    Ag = oracle.assemble(dict(cfg, stabilization=0), z).toarray()
    vel, pr = _blocks(cfg)
    dB, dC = (As - Ag)[np.ix_(vel, pr)], (As - Ag)[np.ix_(pr, vel)]
    assert np.abs(dB).max() > 1e-3
    assert np.abs(dB - dC.T).max() < 1e-14
    D = As[np.ix_(pr, pr)]
    assert np.abs(D - D.T).max() < 1e-14 * np.abs(D).max()


@pytest.mark.parametrize("dim", [2, 3])
def test_aligned_rotation_is_relabeling(dim):
    """Sec. 3.1 rotation: at theta = m dtheta the rotor sits exactly where its
    cells i+m sat at theta = 0, so J(m dtheta; u) = P^T J(0; P u) P with P the
    cyclic relabeling of rotor nodes by m*k positions."""
    k, nt = 2, 6
    cfg0 = _cfg(dim=dim, n_theta=nt, theta_rot=0.0)
    m = 2
    cfgm = dict(cfg0, theta_rot=m * 2 * math.pi / nt)
    n = oracle.n_dofs(cfg0)
    nrot = oracle.sizes(cfg0)[1]
    nc = dim + 1
    ntn = k * nt
    node = np.arange(nrot // nc)
    it = node % ntn
    perm = np.arange(n)
    for c in range(nc):
        perm[node * nc + c] = (node - it + (it + m * k) % ntn) * nc + c
    g = np.random.default_rng(8)
    u, x = g.uniform(-1, 1, n), g.uniform(-1, 1, n)
    Pu, Px = np.empty(n), np.empty(n)
    Pu[perm], Px[perm] = u, x
    y_m = oracle.apply_jacobian(cfgm, u, x)
    y_0 = oracle.apply_jacobian(cfg0, Pu, Px)
    assert np.abs(y_m - y_0[perm]).max() < 1e-13 * np.abs(y_m).max()


def _merge_map(cfg):
    """E: merged conforming DoFs -> mortar DoFs (interface nodes duplicated)."""
    k, nt, dim = cfg["degree"], cfg["n_theta"], cfg["dim"]
    nrr, nrs = k * cfg["n_r_rotor"] + 1, k * cfg["n_r_stator"] + 1
    nzn = k * cfg["n_z"] + 1 if dim == 3 else 1
    ntn, nc = k * nt, dim + 1
    nrg = nrr + nrs - 1
    rows, cols = [], []
    off = ntn * nrr * nzn
    for iz in range(nzn):
        for it in range(ntn):
            for ir in range(nrr):
                rows.append(it + ntn * (ir + nrr * iz))
                cols.append(it + ntn * (ir + nrg * iz))
            for ir in range(nrs):
                rows.append(off + it + ntn * (ir + nrs * iz))
                cols.append(it + ntn * (ir + nrr - 1 + nrg * iz))
    rows, cols = np.array(rows), np.array(cols)
    R = np.concatenate([rows * nc + c for c in range(nc)])
    C = np.concatenate([cols * nc + c for c in range(nc)])
    return sp.csr_matrix((np.ones(R.size), (R, C)), shape=(off * nc + ntn * nrs * nzn * nc, ntn * nrg * nzn * nc))


@pytest.mark.parametrize("dim", [2, 3])
def test_aligned_mortar_reduces_to_conforming_cg(dim):
    """At an aligned angle, E^T J_mortar E equals the stabilized CG operator of
    the merged conforming mesh (the paper's no-mortar reference): for continuous
    fields the jump terms vanish and the two sides' flux terms cancel."""
    cfg = _cfg(dim=dim, theta_rot=0.0)
    cg = dict(cfg, merged=1)
    E = _merge_map(cfg)
    g = np.random.default_rng(9)
    ug = g.uniform(-1, 1, E.shape[1])
    Jm = oracle.assemble(cfg, E @ ug)
    Jg = oracle.assemble(cg, ug)
    free = ~oracle.constrained(cg)
    D = (E.T @ Jm @ E - Jg).toarray()[np.ix_(free, free)]
    assert np.abs(D).max() < 1e-13 * abs(Jg).max()


@pytest.mark.parametrize("dim", [2, 3])
def test_continuity_at_alignment(dim):
    """J(theta) is continuous through an aligned angle: the zero-length segment
    contributes nothing, and the change is linear in the offset."""
    cfg = _cfg(dim=dim, theta_rot=0.0)
    n = oracle.n_dofs(cfg)
    g = np.random.default_rng(10)
    u, x = g.uniform(-1, 1, n), g.uniform(-1, 1, n)
    y0 = oracle.apply_jacobian(cfg, u, x)
    d1 = np.abs(oracle.apply_jacobian(dict(cfg, theta_rot=1e-6), u, x) - y0).max()
    d2 = np.abs(oracle.apply_jacobian(dict(cfg, theta_rot=1e-8), u, x) - y0).max()
    dm = np.abs(oracle.apply_jacobian(dict(cfg, theta_rot=-1e-8), u, x) - y0).max()
    assert d1 < 1e-4 and abs(d1 / d2 - 100) < 1 and dm < 1e-6


# --------------------------------------------------- convergence orders --

def test_pressure_nullspace_up_to_quadrature():
    """Constant pressure is in the nullspace of the unpinned operator (volume
    -(div v, p) against the central flux {p} n) up to Gauss quadrature of the
    polar map, whose error falls as dtheta^(2n) under theta-refinement."""
    errs = []
    for nt in (6, 12, 24):
        cfg = _cfg(n_theta=nt, pin_pressure=0)
        n = oracle.n_dofs(cfg)
        vel, pr = _blocks(cfg)
        x = np.zeros(n)
        x[np.arange(n) % 3 == 2] = 1.0
        u = np.random.default_rng(11).uniform(-1, 1, n)
        errs.append(np.abs(oracle.apply_jacobian(cfg, u, x)[vel | pr]).max())
    r1, r2 = np.log2(errs[0] / errs[1]), np.log2(errs[1] / errs[2])
    assert r1 > 4.5 and r2 > 5.0, errs


def _two_sided_field(cfg, seed):
    """Increment for the mass pin: on each side an independent smooth random
    velocity field (cosine modes of x, y up to wavenumber 2), zero on every
    wall, so that the interface jump is O(1); random smooth pressure."""
    n, n_rot = oracle.sizes(cfg)[:2]
    nc = cfg["dim"] + 1
    X = oracle.node_coords(cfg)
    x, y, z = X[:, 0], X[:, 1], X[:, 2]
    r = np.hypot(x, y)
    rotor = np.arange(n // nc) < n_rot // nc
    wall = np.where(rotor, r - cfg["r_in"], cfg["r_out"] - r)
    if cfg["dim"] == 3:
        wall = wall * z * (cfg["height"] - z)
    g = np.random.default_rng(seed)
    out = np.zeros(n)
    for c in range(nc):
        fr, fs = np.zeros_like(r), np.zeros_like(r)
        for a in range(3):
            for b in range(3):
                cr, cs = g.uniform(-1, 1, 2)
                mode = np.cos(a * np.pi * x + b * np.pi * y + g.uniform(0, 2 * np.pi))
                fr += cr * mode
                fs += cs * mode
        f = np.where(rotor, fr, fs)
        out[c::nc] = f * wall if c < cfg["dim"] else f
    return out


@pytest.mark.parametrize("dim", [2, 3])
def test_discrete_mass_conservation(dim):
    """Eq. EqMortarMass (strong-DG mass term): the sum of all pressure rows of
    J x is the pressure test function q = 1, for which the PSPG term vanishes
    and the volume term integrates div(du) over both domains; by the
    divergence theorem that is the flux through the walls (zero here: x
    vanishes there) plus, on the interface, (du_rotor - du_stator) . e_r,
    which the two sides' mass terms -(1/2) j_s . n_s cancel exactly.  So the
    sum is zero up to the Gauss quadrature of the polar map, whose error falls
    by more than 2^6 per refinement; an O(1) interface jump that the face
    terms did not cancel would stay O(1)."""
    errs, scale = [], []
    for nt in (8, 16, 32):
        c = max(1, nt // 8)
        cfg = _cfg(dim=dim, n_theta=nt, n_r_rotor=c, n_r_stator=c, n_z=c, pin_pressure=0)
        n = oracle.n_dofs(cfg)
        u = np.random.default_rng(3).uniform(-1, 1, n)
        y = oracle.apply_jacobian(cfg, u, _two_sided_field(cfg, 4))
        pr = np.arange(n) % (dim + 1) == dim
        errs.append(abs(y[pr].sum()))
        scale.append(np.abs(y[pr]).max())
    r1, r2 = np.log2(errs[0] / errs[1]), np.log2(errs[1] / errs[2])
    assert r1 > 6.0 and r2 > 6.0, errs
    assert errs[-1] < 1e-8 * scale[-1], (errs, scale)


def _solve_mms(cfg, iters=8):
    import scipy.sparse.linalg as spla

    exact = oracle.mms_interpolate(cfg)
    s = exact.copy()
    for _ in range(iters):
        r = oracle.residual(cfg, s)
        ds = spla.spsolve(oracle.assemble(cfg, s).tocsc(), -r)
        s += ds
        if np.abs(ds).max() < 1e-11:
            break
    return s


@pytest.mark.slow
@pytest.mark.parametrize("theta", [0.0, 0.05])
def test_mms_convergence_q2(theta):
    """Whole discretization, Sec. 4.1: the 2D manufactured solution with nu = 1,
    omega = 0 on the annulus converges at O(h^3) in velocity and O(h^2) in
    pressure (Q2), and the mortar error matches the merged no-mortar mesh."""
    errs = []
    for nt, nr in ((32, 4), (64, 8)):
        cfg = oracle.params(dim=2, degree=2, n_theta=nt, n_r_rotor=nr, n_r_stator=nr, nu=1.0, omega=0.0,
                            theta_rot=theta, mms=1, nthreads=0)
        errs.append(oracle.mms_errors(cfg, _solve_mms(cfg)))
    ru = math.log2(errs[0][0] / errs[1][0])
    rp = math.log2(errs[0][1] / errs[1][1])
    assert ru > 3.0 - 0.25 and rp > 2.0 - 0.25, (ru, rp)
    cg = oracle.params(dim=2, degree=2, n_theta=64, n_r_rotor=8, n_r_stator=8, nu=1.0, omega=0.0, mms=1,
                       merged=1)
    eg = oracle.mms_errors(cg, _solve_mms(cg))
    assert abs(errs[1][0] / eg[0] - 1) < 0.05 and abs(errs[1][1] / eg[1] - 1) < 0.05


@pytest.mark.slow
def test_mms_convergence_q2_unequal_counts():
    """Whole discretization with unequal interface counts (stator rings 3/2 the
    rotor's): the 2D manufactured solution converges at the optimal Q2 rates
    and its error stays within a few percent of the equal-count mesh with
    the same rotor ring."""
    errs = []
    for nt, nr in ((32, 4), (64, 8)):
        cfg = oracle.params(dim=2, degree=2, n_theta=nt, n_theta_stator=3 * nt // 2, n_r_rotor=nr, n_r_stator=nr,
                            nu=1.0, omega=0.0, theta_rot=0.05, mms=1, nthreads=0)
        errs.append(oracle.mms_errors(cfg, _solve_mms(cfg)))
    ru = math.log2(errs[0][0] / errs[1][0])
    rp = math.log2(errs[0][1] / errs[1][1])
    assert ru > 3.0 - 0.25 and rp > 2.0 - 0.25, (ru, rp)
    ce = oracle.params(dim=2, degree=2, n_theta=64, n_r_rotor=8, n_r_stator=8, nu=1.0, omega=0.0,
                       theta_rot=0.05, mms=1)
    ee = oracle.mms_errors(ce, _solve_mms(ce))
    print(errs, ee)
    assert errs[1][0] < 1.5 * ee[0] and errs[1][1] < 1.5 * ee[1]


@pytest.mark.slow
def test_mms_convergence_q3():
    """As above for Q3: O(h^4) velocity, O(h^3) pressure (pre-asymptotic on
    these meshes, so the bound is one order lower than Q3's optimum minus a
    margin, and strictly above the Q2 optimum for velocity)."""
    errs = []
    for nt, nr in ((16, 2), (32, 4)):
        cfg = oracle.params(dim=2, degree=3, n_theta=nt, n_r_rotor=nr, n_r_stator=nr, nu=1.0, omega=0.0,
                            theta_rot=0.03, mms=1)
        errs.append(oracle.mms_errors(cfg, _solve_mms(cfg)))
    ru = math.log2(errs[0][0] / errs[1][0])
    rp = math.log2(errs[0][1] / errs[1][1])
    assert ru > 3.3 and rp > 2.5, (ru, rp)


_TGV_KAPPA = math.pi


def _tgv_levels(cfg, t, nu):
    """Taylor-Green vortex of wavenumber kappa at the nodes of cfg (rotor nodes
    at cfg's rotor angle), velocity and pressure interleaved:
    u = (sin kx cos ky, -cos kx sin ky) F, p = (cos 2kx + cos 2ky) F^2 / 4,
    F = exp(-2 nu k^2 t).  (u.grad)u + grad p = 0 and du/dt = nu lap u, so it
    solves the incompressible equations exactly (decay e^{-4 nu k^2 t} of the
    pressure included)."""
    kap = _TGV_KAPPA
    xyz = oracle.node_coords(cfg)
    x, y = xyz[:, 0], xyz[:, 1]
    f = math.exp(-2.0 * nu * kap * kap * t)
    out = np.empty(3 * len(x))
    out[0::3] = np.sin(kap * x) * np.cos(kap * y) * f
    out[1::3] = -np.cos(kap * x) * np.sin(kap * y) * f
    out[2::3] = 0.25 * (np.cos(2 * kap * x) + np.cos(2 * kap * y)) * f * f
    return out


def _tgv_run(n_theta, n_r_rotor, n_r_stator, dt, t_end, omega, nu=0.05, theta0=0.2):
    """BDF2 + Newton on the oracle's transient residual (Sec. 2.2 time
    discretization, Sec. 3.1 rotating rotor): the rotor advances omega dt per
    step, the walls and the pinned pressure take the exact values of the new
    level, the two start levels are exact.  Returns the relative max-norm
    errors of velocity and pressure at t_end."""
    import scipy.sparse.linalg as spla

    base = dict(dim=2, degree=2, r_in=0.3, r_if=0.55, r_out=1.0, n_theta=n_theta, n_r_rotor=n_r_rotor,
                n_r_stator=n_r_stator, nu=nu, steady=0, dt=dt, omega=omega, nthreads=0)

    def cfg(step):
        return oracle.params(**base, theta_rot=theta0 + omega * step * dt)

    cons = oracle.constrained(cfg(0))
    levels = [_tgv_levels(cfg(-1), -dt, nu), _tgv_levels(cfg(0), 0.0, nu)]
    nsteps = int(round(t_end / dt))
    for step in range(1, nsteps + 1):
        c = cfg(step)
        exact = _tgv_levels(c, step * dt, nu)
        hist = (levels[-2] - 4.0 * levels[-1]) / (2.0 * dt)
        u = levels[-1].copy()
        u[cons] = exact[cons]
        for _ in range(20):
            r = oracle.residual(c, u, hist)
            if np.abs(r).max() < 1e-12:
                break
            u += spla.spsolve(oracle.assemble(c, u, hist).tocsc(), -r)
        else:
            raise AssertionError("Newton did not converge on the Taylor-Green step")
        levels.append(u)
    return _tgv_errors(levels[-1], exact)


def _tgv_errors(u, exact):
    vel = np.arange(len(u)) % 3 != 2
    e = np.abs(u - exact)
    return e[vel].max() / np.abs(exact[vel]).max(), e[~vel].max() / np.abs(exact[~vel]).max()


@pytest.mark.slow
def test_taylor_green_transient_with_rotating_rotor():
    """Transient path end to end on an exact solution: the Taylor-Green vortex
    is a solution in the laboratory frame whatever the mesh does, so with the
    rotor turning (omega = 1, mortar at a new angle every step, ALE convection
    and BDF2 on material-frame nodal values) the error must match the fixed
    rotor's and fall with h and dt halved at the rate of Q2 in space and BDF2
    in time (measured: velocity 14.8e-3 -> 1.18e-3, pressure 0.123 -> 0.023)."""
    coarse = (16, 2, 3, 0.1)
    fine = (32, 4, 6, 0.05)
    ev0, ep0 = _tgv_run(*fine, 0.4, 0.0)
    ev_c, ep_c = _tgv_run(*coarse, 0.4, 1.0)
    ev_f, ep_f = _tgv_run(*fine, 0.4, 1.0)
    assert math.log2(ev_c / ev_f) > 3.0, (ev_c, ev_f)
    assert math.log2(ep_c / ep_f) > 2.0, (ep_c, ep_f)
    assert ev_f < 2e-3 and ep_f < 3e-2, (ev_f, ep_f)
    assert abs(ev_f / ev0 - 1.0) < 0.1 and abs(ep_f / ep0 - 1.0) < 0.1, (ev_f, ev0, ep_f, ep0)
