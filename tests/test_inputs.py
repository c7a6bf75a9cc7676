"""Seeded input recipes (CPU): the workloads and the batching instances have
the stated sizes, ranges and determinism."""
import math

import numpy as np

from paper_2608_27423_amd import inputs


def test_workload_dof_counts():
    expect = {"annulus2d_q2_32x4": 3456, "annulus3d_q2_64x8x32": 1131520, "annulus3d_q3_64x16x32": 7300608,
              "annulus3d_q2_256x32x128": 68423680}
    for name, n in expect.items():
        assert inputs.n_dofs(inputs.mesh(name)) == n


def test_batch_instances_recipe():
    a = inputs.batch_instances()
    b = inputs.batch_instances()
    assert len(a) == 48
    assert [(m["n_theta"], th) for m, th, _, _ in a] == [(m["n_theta"], th) for m, th, _, _ in b]
    dims = [m["dim"] for m, _, _, _ in a]
    assert dims.count(2) == 24 and dims.count(3) == 24
    res = []
    for m, th, om, seed in a:
        assert 0.0 <= th < 2 * math.pi and om == 1.0
        assert m["degree"] == 2 and m["steady"] == 1
        if m["dim"] == 2:
            assert (m["n_theta"], m["n_r_rotor"]) in inputs.BATCH_SIZES_2D
        else:
            assert (m["n_theta"], m["n_r_rotor"], m["n_z"]) in inputs.BATCH_SIZES_3D
        assert m["n_r_rotor"] == m["n_r_stator"]
        res.append(1.0 / m["nu"])
    assert 1.0 <= min(res) and max(res) <= 2000.0
    # log-uniform: the logs spread over most of [0, log 2000]
    lr = np.log(res)
    assert lr.max() - lr.min() > 0.6 * math.log(2000.0)
    # uneven sizes: at least three distinct sizes per dimension
    assert len({(m["n_theta"], m["n_r_rotor"]) for m, _, _, _ in a if m["dim"] == 2}) >= 3
    assert len({(m["n_theta"], m["n_z"]) for m, _, _, _ in a if m["dim"] == 3}) >= 3


def test_transient_start_satisfies_dirichlet_data():
    m = inputs.mesh("annulus3d_q2_64x8x32", n_theta=8, n_r_rotor=2, n_r_stator=2, n_z=2)
    u = inputs.transient_start(m, 5)
    ntn, nrr, nrs, nzn = inputs.node_grid(m)
    v = u.reshape(-1, 4)
    rot = v[: ntn * nrr * nzn].reshape(nzn, nrr, ntn, 4)
    sta = v[ntn * nrr * nzn:].reshape(nzn, nrs, ntn, 4)
    assert np.abs(u).max() <= 1.0 + 1e-15
    assert np.all(rot[:, 0, :, :3] == 0) and np.all(sta[:, -1, :, :3] == 0)
    assert np.all(rot[0, :, :, :3] == 0) and np.all(sta[-1, :, :, :3] == 0)
    assert sta[0, -1, 0, 3] == 0
