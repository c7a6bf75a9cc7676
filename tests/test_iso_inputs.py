"""The curved-mesh node recipe of inputs.iso_node_positions (the GPU tests'
input) against the oracle's own iso-parametric node positions: the oracle
builds its mesh from orc_params.iso / perturb alone, so agreement pins that
both sides integrate over the same cells.  Also: the Gauss-Lobatto nodes of
inputs against the oracle's rules, and the rigid rotor rotation."""
import math

import numpy as np
import pytest

import oracle
from helpers import oracle_cfg, small_mesh
from paper_2608_27423_amd import inputs


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5])
def test_lobatto_nodes_match_oracle_rules(k):
    gll = np.asarray(oracle.rules(k + 1)[0])
    assert np.abs(inputs.lobatto_nodes(k) - gll).max() <= 1e-15


@pytest.mark.parametrize("dim,k,kw", [(2, 2, {}), (2, 5, {}), (3, 2, {}), (3, 3, dict(n_theta_stator=7)),
                                      (3, 4, dict(n_theta=4))])
@pytest.mark.parametrize("perturb", [0.0, 0.1])
def test_iso_nodes_match_oracle(dim, k, kw, perturb):
    mesh = small_mesh(dim, k, **kw)
    x0 = inputs.iso_node_positions(mesh, perturb)
    for theta in (0.0, 2.1):
        xo = np.asarray(oracle.node_coords(oracle_cfg(mesh, theta, 1.0, iso=1, perturb=perturb))).reshape(-1, 3)
        x = inputs.rotate_rotor_nodes(mesh, x0, theta)
        assert x.shape == xo.shape
        assert np.abs(x - xo).max() <= 1e-14


def test_iso_nodes_keep_walls_and_interface():
    mesh = small_mesh(3, 3)
    x = inputs.iso_node_positions(mesh, 0.2)
    ntn, nrr, nrs, nzn = inputs.node_grid(mesh)
    r = np.hypot(x[:, 0], x[:, 1])
    rot = r[: ntn * nrr * nzn].reshape(nzn, nrr, ntn)
    sta = r[ntn * nrr * nzn:].reshape(nzn, nrs, ntn)
    assert np.abs(rot[:, 0] - mesh["r_in"]).max() < 1e-14
    assert np.abs(rot[:, -1] - mesh["r_if"]).max() < 1e-14
    assert np.abs(sta[:, 0] - mesh["r_if"]).max() < 1e-14
    assert np.abs(sta[:, -1] - mesh["r_out"]).max() < 1e-14
    # interior nodes do move, by a fraction of a cell
    dr_c = max((mesh["r_if"] - mesh["r_in"]) / mesh["n_r_rotor"], (mesh["r_out"] - mesh["r_if"]) / mesh["n_r_stator"])
    polar = np.hypot(*inputs.iso_node_positions(mesh, 0.0)[:, :2].T)
    moved = np.abs(r - polar)
    assert 0.05 * dr_c < moved.max() <= 0.2 * dr_c * (1 + 1e-12)


def test_rotate_rotor_nodes():
    mesh = small_mesh(2, 2)
    x = inputs.iso_node_positions(mesh, 0.1)
    y = inputs.rotate_rotor_nodes(mesh, x, math.pi / 2)
    ntn, nrr, _, _ = inputs.node_grid(mesh)
    n_rot = ntn * nrr
    assert np.allclose(y[:n_rot, 0], -x[:n_rot, 1], atol=1e-15) and np.allclose(y[:n_rot, 1], x[:n_rot, 0], atol=1e-15)
    assert np.array_equal(y[n_rot:], x[n_rot:])
