"""Preconditioner replayed from a HIP graph (mns_solve_opts.use_graph) against
the same solve launched kernel by kernel: the same kernels run in the same
order on the same buffers, so iteration counts and solutions agree exactly
(also for the single-level polynomials, which stop at the iteration limit on
this transient operator; the V-cycle converges).
Covers the Chebyshev polynomials in FP32 and FP64, the V-cycle in both
precisions, and the concurrent mortar launch (second stream joined inside the
captured graph); two solves in a row on one handle rebuild the graph."""
import numpy as np
import pytest

from paper_2608_27423_amd import binding, inputs
from tests.helpers import small_mesh

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=torch.float64)


@pytest.mark.parametrize("fused", [1, 2])
@pytest.mark.parametrize("precond", ["f32", "f64", "mg", "mg64"])
def test_graph_replay_matches_eager_solve(precond, fused):
    mesh = small_mesh(3, 2, n_theta=16, n_r_rotor=4, n_r_stator=4, n_z=4, steady=0, dt=0.02, nu=0.005)
    n = inputs.n_dofs(mesh)
    g = np.random.default_rng(77)
    state = inputs.transient_start(mesh, 78)
    hist = g.uniform(-1, 1, n)
    rhs = [g.uniform(-1, 1, n), g.uniform(-1, 1, n)]
    out = {}
    with binding.Operator(mesh) as op:
        op.set_kernel_config(fused_launch=fused)
        op.rotate_rotor(0.9, 0.7)
        op.set_linearization(_dev(state), _dev(hist))
        for use_graph in (1, 0):
            res = []
            for b in rhs:  # two solves in a row: the graph is built per call
                x = torch.zeros(n, dtype=torch.float64, device="cuda")
                _, rep = op.solve(_dev(b), x, check=False, rtol=1e-10, restart=60, maxit=150, precond=precond,
                                  use_graph=use_graph)
                res.append((rep, x.cpu().numpy()))
            out[use_graph] = res
    for (rg, xg), (re, xe) in zip(out[1], out[0]):
        print(f"{precond} fused={fused}: its graph {rg['iterations']} eager {re['iterations']}, "
              f"{rg['seconds'] * 1e3:.1f} ms vs {re['seconds'] * 1e3:.1f} ms")
        assert rg["rc"] == re["rc"]
        assert precond in ("f32", "f64") or rg["rc"] == 0
        assert rg["iterations"] == re["iterations"]
        assert rg["vmults_f64"] == re["vmults_f64"] and rg["vmults_f32"] == re["vmults_f32"]
        assert np.array_equal(xg, xe)
