"""Batches with curved (iso-parametric) instances: each (dimension, degree)
of curved instances is a launch group of its own, running the blocks of the
single-instance curved fused launch, so every curved slice equals the
instance's own product bit for bit (FP64 and FP32) and the oracle's curved
product to the parity bar; polar instances of the same dimension and degree
in the same batch keep theirs.  Batched solves (Jacobi-Chebyshev and the
V-cycle with curved coarse levels) take the single solves' iteration
counts."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla
import torch

import oracle
from helpers import oracle_cfg, relmax, small_mesh
from paper_2608_27423_amd import binding, inputs

pytestmark = pytest.mark.gpu

PERT = 0.1


def _dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def test_batch_curved_and_polar_instances_equal_single_applications():
    # (dim, k, curved, mesh keywords)
    kinds = [(2, 2, True, dict(n_theta=12)), (3, 2, True, dict(n_theta=16, n_z=2)), (3, 2, False, dict(n_theta=16)),
             (2, 3, True, dict(n_theta=7)), (3, 3, True, dict(n_theta=8, n_z=2)), (2, 2, False, dict(n_theta=7)),
             (3, 4, True, dict(n_theta=4, n_r_rotor=1, n_r_stator=1, n_z=1)), (3, 2, True, dict(n_theta=5))]
    g = np.random.default_rng(31)
    ops, cfgs, states, hists = [], [], [], []
    try:
        for j, (dim, k, curved, kw) in enumerate(kinds):
            mesh = small_mesh(dim, k, nu=0.01 * (1 + j), steady=j % 2, dt=0.05, **kw)
            theta, omega = 0.4 + 0.8 * j, 0.9
            op = binding.Operator(mesh)
            if curved:
                op.set_node_positions(inputs.iso_node_positions(mesh, PERT))
            op.rotate_rotor(theta, omega)
            state = g.uniform(-1, 1, op.n_dofs)
            hist = None if mesh["steady"] else g.uniform(-1, 1, op.n_dofs)
            op.set_linearization(_dev(state), None if hist is None else _dev(hist))
            ops.append(op)
            states.append(state)
            hists.append(hist)
            cfgs.append(oracle_cfg(mesh, theta, omega, iso=1, perturb=PERT) if curved
                        else oracle_cfg(mesh, theta, omega))
        with binding.Batch(ops) as b:
            x = g.uniform(-1, 1, b.n_dofs)
            y64 = b.apply_jacobian(_dev(x)).cpu().numpy()
            y32 = b.apply_jacobian(_dev(x, torch.float32)).cpu().numpy()
            for i, op in enumerate(ops):
                sl = slice(b.offsets[i], b.offsets[i] + op.n_dofs)
                op.set_kernel_config(fused_launch=1)
                s64 = op.apply_jacobian(_dev(x[sl])).cpu().numpy()
                s32 = op.apply_jacobian(_dev(x[sl], torch.float32)).cpu().numpy()
                assert np.array_equal(y64[sl], s64), f"instance {i} FP64"
                assert np.array_equal(y32[sl], s32), f"instance {i} FP32"
                err = relmax(y64[sl], oracle.apply_jacobian(cfgs[i], states[i], x[sl], hist=hists[i]))
                print(f"instance {i} {kinds[i][:3]} ({op.n_dofs} DoFs): fp64 vs oracle {err:.2e}")
                assert err <= 1e-12
            # a rotation of a curved member is seen by the batch (its metric
            # and mortar point tables are recomputed in place)
            ops[1].rotate_rotor(2.0, 0.3)
            ops[1].set_linearization(_dev(states[1]), None if hists[1] is None else _dev(hists[1]))
            y64b = b.apply_jacobian(_dev(x)).cpu().numpy()
            sl = slice(b.offsets[1], b.offsets[1] + ops[1].n_dofs)
            assert np.array_equal(y64b[sl], ops[1].apply_jacobian(_dev(x[sl])).cpu().numpy())
    finally:
        for op in ops:
            op.close()


@pytest.mark.parametrize("precond", ["f32", "mg"])
def test_batch_solve_curved_instances(precond):
    """A batched solve over curved 2D and 3D instances (and one polar one)
    gives each instance its single solve's iteration count within two and the
    oracle's direct solution of its curved Jacobian."""
    sizes = [(2, 2, dict(n_theta=16, n_r_rotor=4, n_r_stator=4)), (3, 2, dict(n_theta=16, n_r_stator=2, n_z=2)),
             (3, 3, dict(n_theta=8, n_r_rotor=1, n_r_stator=1, n_z=1)),
             (2, 2, dict(n_theta=16, n_r_rotor=2, n_r_stator=2))]
    g = np.random.default_rng(47)
    ops, rhs, direct = [], [], []
    try:
        for j, (dim, k, kw) in enumerate(sizes):
            curved = j < 3
            mesh = small_mesh(dim, k, steady=0, dt=0.05, nu=0.05 * (1 + 0.3 * j), **kw)
            theta, omega = 0.5 + 1.1 * j, 0.7
            sm = inputs.smooth_field(mesh, 60 + j)
            state = 0.5 * sm / np.abs(sm).max()
            hist = g.uniform(-1, 1, inputs.n_dofs(mesh))
            op = binding.Operator(mesh)
            if curved:
                op.set_node_positions(inputs.iso_node_positions(mesh, PERT))
            op.rotate_rotor(theta, omega)
            op.set_linearization(_dev(state), _dev(hist))
            ops.append(op)
            b = g.uniform(-1, 1, op.n_dofs)
            rhs.append(b)
            cfg = oracle_cfg(mesh, theta, omega, iso=1, perturb=PERT) if curved else oracle_cfg(mesh, theta, omega)
            direct.append(spla.spsolve(oracle.assemble(cfg, state, hist).tocsc(), b))
        opts = dict(rtol=1e-10, restart=30, maxit=3000, precond=precond)
        if precond == "f32":
            opts["cheb_degree"] = 6
        with binding.Batch(ops) as bt:
            x, rc, reps = bt.solve(_dev(np.concatenate(rhs)), check=False, **opts)
            assert rc == 0, bt.last_error()
            xb = x.cpu().numpy()
            for i, op in enumerate(ops):
                _, rep1 = op.solve(_dev(rhs[i]), check=False, **opts)
                err = relmax(xb[bt.offsets[i]:bt.offsets[i] + op.n_dofs], direct[i])
                print(f"{precond} instance {i}: batch its {reps[i]['iterations']} (single {rep1['iterations']}), "
                      f"|x - x_direct| / |x| = {err:.1e}")
                assert reps[i]["status"] == 0 and rep1["rc"] == 0
                assert err < 1e-8
                assert abs(reps[i]["iterations"] - rep1["iterations"]) <= 2
    finally:
        for op in ops:
            op.close()
