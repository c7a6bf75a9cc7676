"""Named workloads and seeded synthetic inputs.

This module is shared by the HIP path's tests/benchmark and by the oracle's
tests.  It holds no arithmetic of the method: only mesh descriptions, seeded
random numbers (numpy PCG64) and smooth synthetic fields defined on the DoF
index grid.  The paper's own meshes, CAD geometries and measured data are not
available; these annular rotor/stator meshes stand in for them.
"""
import math

import numpy as np

TWO_PI = 2.0 * math.pi

# Annular rotor/stator workloads.  Cell counts are per domain
# (n_theta azimuthal x n_r radial [x n_z axial]).
WORKLOADS = {
    "annulus2d_q2_32x4": dict(
        dim=2, degree=2, r_in=0.25, r_if=0.5, r_out=1.0, height=1.0, n_theta=32, n_r_rotor=4,
        n_r_stator=4, n_z=1, nu=0.01, omega=1.0, steady=1, dt=1.0),
    "annulus3d_q2_64x8x32": dict(
        dim=3, degree=2, r_in=0.2, r_if=0.5, r_out=1.0, height=1.0, n_theta=64, n_r_rotor=8,
        n_r_stator=8, n_z=32, nu=0.01, omega=1.0, steady=1, dt=1.0),
    "annulus3d_q3_64x16x32": dict(
        dim=3, degree=3, r_in=0.2, r_if=0.5, r_out=1.0, height=1.0, n_theta=64, n_r_rotor=16,
        n_r_stator=16, n_z=32, nu=0.005, omega=1.0, steady=1, dt=1.0),
    "annulus3d_q2_256x32x128": dict(
        dim=3, degree=2, r_in=0.2, r_if=0.5, r_out=1.0, height=1.0, n_theta=256, n_r_rotor=32,
        n_r_stator=32, n_z=128, nu=5e-4, omega=1.0, steady=0, dt=0.01),
}

# rotor angle of each workload: fixed 0.1 rad for the 2D case, seeded otherwise
ANGLE_SEED = {"annulus3d_q2_64x8x32": 2, "annulus3d_q3_64x16x32": 6, "annulus3d_q2_256x32x128": 11}
STATE_SEED = {"annulus2d_q2_32x4": 0, "annulus3d_q2_64x8x32": 3, "annulus3d_q3_64x16x32": 7,
              "annulus3d_q2_256x32x128": 12}
VECTOR_SEED = {"annulus2d_q2_32x4": 1, "annulus3d_q2_64x8x32": 4, "annulus3d_q3_64x16x32": 8,
               "annulus3d_q2_256x32x128": 13}
SOLUTION_SEED = {"annulus2d_q2_32x4": 14, "annulus3d_q2_64x8x32": 5, "annulus3d_q3_64x16x32": 9,
                 "annulus3d_q2_256x32x128": 15}


def mesh(name, **overrides):
    m = dict(WORKLOADS[name])
    m.update(overrides)
    return m


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def uniform(n, seed, lo=-1.0, hi=1.0):
    """n values uniform in [lo, hi) from PCG64(seed)."""
    return rng(seed).uniform(lo, hi, n)


def rotor_angle(name):
    if name == "annulus2d_q2_32x4":
        return 0.1
    return float(rng(ANGLE_SEED[name]).uniform(0.0, TWO_PI))


def node_grid(m):
    """Per-direction node counts: (k*n_theta, k*n_r_rotor+1, k*n_r_stator+1, k*n_z+1 or 1)."""
    k = m["degree"]
    nzn = k * m["n_z"] + 1 if m["dim"] == 3 else 1
    return k * m["n_theta"], k * m["n_r_rotor"] + 1, k * m["n_r_stator"] + 1, nzn


def n_dofs(m):
    ntn, nrr, nrs, nzn = node_grid(m)
    nts = m["degree"] * m["n_theta_stator"] if m.get("n_theta_stator") else ntn  # stator ring, when it differs
    return (ntn * nrr + nts * nrs) * nzn * (m["dim"] + 1)


def _index_coords(m):
    """Approximate node positions from the node indices alone (theta, r, z equally
    spaced per domain, rotor at zero angle); smooth-field inputs only."""
    ntn, nrr, nrs, nzn = node_grid(m)
    nts = m["degree"] * m["n_theta_stator"] if m.get("n_theta_stator") else ntn
    out = []
    for nt_nodes, nr_nodes, r0, r1 in ((ntn, nrr, m["r_in"], m["r_if"]), (nts, nrs, m["r_if"], m["r_out"])):
        th = TWO_PI * np.arange(nt_nodes) / nt_nodes
        r = np.linspace(r0, r1, nr_nodes)
        z = np.linspace(0.0, m["height"], nzn) if m["dim"] == 3 else np.zeros(1)
        Z, R, T = np.meshgrid(z, r, th, indexing="ij")
        out.append((R * np.cos(T)).ravel())
        out.append((R * np.sin(T)).ravel())
        out.append(Z.ravel())
    x = np.concatenate([out[0], out[3]])
    y = np.concatenate([out[1], out[4]])
    z = np.concatenate([out[2], out[5]])
    return x, y, z


def smooth_field(m, seed, max_wavenumber=3):
    """Every component = sum over m, n <= max_wavenumber of
    A cos(m pi x) cos(n pi y) + B sin sin + C cos sin + D sin cos, coefficients
    uniform in [-1, 1] (PCG64(seed)); in 3D multiplied by a z series
    sum_l E_l cos(l pi z) + F_l sin(l pi z).  Returned in DoF layout."""
    x, y, z = _index_coords(m)
    nc = m["dim"] + 1
    g = rng(seed)
    K = max_wavenumber + 1
    out = np.empty((x.size, nc))
    pix, piy, piz = math.pi * x, math.pi * y, math.pi * z
    cx = [np.cos(i * pix) for i in range(K)]
    sx = [np.sin(i * pix) for i in range(K)]
    cy = [np.cos(i * piy) for i in range(K)]
    sy = [np.sin(i * piy) for i in range(K)]
    for comp in range(nc):
        coef = g.uniform(-1.0, 1.0, (K, K, 4))
        f = np.zeros_like(x)
        for i in range(K):
            for j in range(K):
                A, B, C, D = coef[i, j]
                f += A * cx[i] * cy[j] + B * sx[i] * sy[j] + C * cx[i] * sy[j] + D * sx[i] * cy[j]
        if m["dim"] == 3:
            zc = g.uniform(-1.0, 1.0, (K, 2))
            fz = np.zeros_like(z)
            for l in range(K):
                fz += zc[l, 0] * np.cos(l * piz) + zc[l, 1] * np.sin(l * piz)
            f *= fz
        out[:, comp] = f
    return out.ravel()


def state_for(name):
    """Linearization state of a workload: smooth manufactured field for the 2D
    case, nodal uniform [-1, 1] otherwise."""
    m = WORKLOADS[name]
    if name == "annulus2d_q2_32x4":
        return smooth_field(m, STATE_SEED[name])
    return uniform(n_dofs(m), STATE_SEED[name])


def vector_for(name):
    return uniform(n_dofs(WORKLOADS[name]), VECTOR_SEED[name])


def transient_start(m, seed):
    """Start level of a transient run: the smooth field scaled to max |.| = 1
    with the no-slip walls (r_in, r_out and, in 3D, z = 0 and z = H) and the
    pinned pressure node (stator, theta index 0, outermost ring, z index 0)
    set to zero, so that it satisfies the Dirichlet data of the problem."""
    u = smooth_field(m, seed)
    u /= np.abs(u).max()
    ntn, nrr, nrs, nzn = node_grid(m)
    nc = m["dim"] + 1
    v = u.reshape(-1, nc)
    rot = v[: ntn * nrr * nzn].reshape(nzn, nrr, ntn, nc)
    sta = v[ntn * nrr * nzn:].reshape(nzn, nrs, ntn, nc)
    rot[:, 0, :, : m["dim"]] = 0.0
    sta[:, -1, :, : m["dim"]] = 0.0
    if m["dim"] == 3:
        for blk in (rot, sta):
            blk[0, :, :, : m["dim"]] = 0.0
            blk[-1, :, :, : m["dim"]] = 0.0
    sta[0, -1, 0, m["dim"]] = 0.0
    return u


# Batching workload: uneven rotor/stator instances of the 2D and 3D Q2 forms
BATCH_SIZES_2D = [(32, 4), (64, 8), (128, 16), (256, 32)]          # n_theta x n_r per domain
BATCH_SIZES_3D = [(16, 4, 8), (32, 4, 8), (32, 8, 16), (64, 8, 16)]  # n_theta x n_r x n_z per domain


def batch_instances(count=48, seed=21):
    """`count` instances, half 2D and half 3D Q2, mesh sizes drawn uniformly
    from the lists above, rotor angle uniform in [0, 2 pi), Reynolds number
    log-uniform in [1, 2000] (nu = 1 / Re, steady).  Returns a list of
    (mesh, theta, omega, state seed)."""
    g = rng(seed)
    out = []
    for i in range(count):
        if i % 2 == 0:
            nt, nr = BATCH_SIZES_2D[int(g.integers(len(BATCH_SIZES_2D)))]
            m = mesh("annulus2d_q2_32x4", n_theta=nt, n_r_rotor=nr, n_r_stator=nr)
        else:
            nt, nr, nz = BATCH_SIZES_3D[int(g.integers(len(BATCH_SIZES_3D)))]
            m = mesh("annulus3d_q2_64x8x32", n_theta=nt, n_r_rotor=nr, n_r_stator=nr, n_z=nz)
        re = float(np.exp(g.uniform(0.0, np.log(2000.0))))
        m["nu"] = 1.0 / re
        out.append((m, float(g.uniform(0.0, TWO_PI)), 1.0, 100 + i))
    return out


def lobatto_nodes(k):
    """The k + 1 Gauss-Lobatto nodes on [0, 1] (0, the roots of P_k', 1): where
    a degree-k cell has its nodes along each direction."""
    inner = np.sort(np.polynomial.legendre.Legendre.basis(k).deriv().roots().real)
    return np.concatenate([[0.0], 0.5 * (inner + 1.0), [1.0]])


def iso_node_positions(m, perturb):
    """Node positions of a curved (iso-parametric) mesh: every Gauss-Lobatto
    node of the annular mesh, at polar position (r, theta_m, z) in the
    material frame, moved by
        dr     = e dr_c  s cos(3 theta_m + 2 pi z / H)
        dtheta = e dth_c s sin(2 theta_m) (1 + cos(2 pi z / H) / 2)
        dz     = e dz_c  s sin(theta_m) sin(pi z / H)        (3D)
    with e = perturb, dr_c, dth_c, dz_c the cell sizes of the node's domain and
    s = sin(pi (r - r_a) / (r_b - r_a)) on that domain [r_a, r_b], so that the
    nodes of the walls and of the interface keep their radius and angle.
    Returns an (n_nodes, 3) array in the node order of the vector layout,
    rotor nodes unrotated (z = 0 in 2D)."""
    k, dim = m["degree"], m["dim"]
    g = lobatto_nodes(k)
    nz = m["n_z"] if dim == 3 else 1
    H = m["height"] if dim == 3 else 1.0
    dz_c = H / nz
    nts = m.get("n_theta_stator") or m["n_theta"]
    out = []
    for nt, nr, ra, rb in ((m["n_theta"], m["n_r_rotor"], m["r_in"], m["r_if"]),
                           (nts, m["n_r_stator"], m["r_if"], m["r_out"])):
        dth_c, dr_c = TWO_PI / nt, (rb - ra) / nr
        it = np.arange(k * nt)
        ir = np.arange(k * nr + 1)
        iz = np.arange(k * nz + 1) if dim == 3 else np.zeros(1, dtype=int)
        th = (it // k + g[it % k]) * dth_c
        r = ra + (ir // k + g[ir % k]) * dr_c
        z = (iz // k + g[iz % k]) * dz_c if dim == 3 else np.zeros(1)
        Z, R, T = np.meshgrid(z, r, th, indexing="ij")
        s = np.sin(math.pi * (R - ra) / (rb - ra))
        zr = 2.0 * math.pi * Z / H if dim == 3 else np.zeros_like(Z)
        rr = R + perturb * dr_c * s * np.cos(3.0 * T + zr)
        tt = T + perturb * dth_c * s * np.sin(2.0 * T) * (1.0 + 0.5 * np.cos(zr))
        zz = Z + (perturb * dz_c * s * np.sin(T) * np.sin(math.pi * Z / H) if dim == 3 else 0.0)
        out.append(np.stack([(rr * np.cos(tt)).ravel(), (rr * np.sin(tt)).ravel(), np.broadcast_to(zz, rr.shape).ravel()],
                            axis=1))
    return np.concatenate(out, axis=0)


def rotate_rotor_nodes(m, xyz, theta):
    """Node positions with the rotor block rotated by theta about the z axis
    (x = R(theta) x0): the current configuration of the mesh."""
    ntn, nrr, _, nzn = node_grid(m)
    n_rot = ntn * nrr * nzn
    out = np.array(xyz, dtype=np.float64, copy=True)
    c, s = math.cos(theta), math.sin(theta)
    x, y = out[:n_rot, 0].copy(), out[:n_rot, 1].copy()
    out[:n_rot, 0] = c * x - s * y
    out[:n_rot, 1] = s * x + c * y
    return out
