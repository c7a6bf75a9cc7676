"""Stream ordering of the boundary calls.

mns_rotate_rotor builds its tables with one kernel on the caller's stream, and
mns_set_linearization / mns_apply_jacobian allocate nothing, so the sequence
rotate -> linearize -> apply behaves the same on a non-default torch stream
and inside a stream capture (replayed several times, with other eager work on
the same handle between the replays) as when launched eagerly on the default
stream.  Results are compared bit for bit: the same kernels run on the same
inputs in every case.  Also: a batch whose member was rotated after the batch
was created refuses to apply or solve until that member is relinearized."""
import numpy as np
import pytest

from paper_2608_27423_amd import binding, inputs
from tests.helpers import small_mesh

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=torch.float64)


def _eager(op, theta, omega, state, x):
    op.rotate_rotor(theta, omega)
    op.set_linearization(state)
    y = op.apply_jacobian(x)
    torch.cuda.synchronize()
    return y.cpu().numpy()


@pytest.mark.parametrize("dim", [2, 3])
def test_rotate_apply_on_side_stream(dim):
    mesh = small_mesh(dim, 2, n_theta=16, n_r_rotor=2, n_r_stator=2, n_z=2)
    n = inputs.n_dofs(mesh)
    state, x = _dev(inputs.uniform(n, 31)), _dev(inputs.uniform(n, 32))
    with binding.Operator(mesh) as op:
        ref = {th: _eager(op, th, 0.8, state, x) for th in (0.37, 2.9)}
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            got = {}
            for th in (2.9, 0.37, 2.9):  # each rotation rewrites the tables in stream order
                op.rotate_rotor(th, 0.8)
                op.set_linearization(state)
                got[th] = op.apply_jacobian(x).clone()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        for th in (0.37, 2.9):
            print(f"dim={dim} theta={th}: side stream == default stream")
            assert np.array_equal(got[th].cpu().numpy(), ref[th])


@pytest.mark.parametrize("fused", [1, 2])
@pytest.mark.parametrize("dim", [2, 3])
def test_rotate_apply_in_graph_capture(dim, fused):
    mesh = small_mesh(dim, 2, n_theta=16, n_r_rotor=2, n_r_stator=3, n_z=2)
    n = inputs.n_dofs(mesh)
    state, x = _dev(inputs.uniform(n, 41)), _dev(inputs.uniform(n, 42))
    theta, other = 1.234, 4.5
    with binding.Operator(mesh) as op:
        op.set_kernel_config(fused_launch=fused)
        ref = _eager(op, theta, 1.1, state, x)
        ref_other = _eager(op, other, 1.1, state, x)
        y = torch.empty_like(x)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            op.rotate_rotor(theta, 1.1)
            op.set_linearization(state)
            op.apply_jacobian(x, y)
        torch.cuda.synchronize()
        for rep in range(3):
            # eager work on the same handle between replays: another angle
            y_other = _eager(op, other, 1.1, state, x)
            assert np.array_equal(y_other, ref_other)
            y.fill_(0.0)
            g.replay()
            torch.cuda.synchronize()
            print(f"dim={dim} fused={fused} replay {rep}: equal to eager")
            assert np.array_equal(y.cpu().numpy(), ref)
        del g


def test_batch_refuses_stale_member():
    mesh = small_mesh(2, 2, n_theta=8)
    n = inputs.n_dofs(mesh)
    ops = [binding.Operator(mesh) for _ in range(2)]
    try:
        for i, op in enumerate(ops):
            op.rotate_rotor(0.3 + i, 1.0)
            op.set_linearization(_dev(inputs.uniform(n, 50 + i)))
        with binding.Batch(ops) as b:
            x = _dev(inputs.uniform(b.n_dofs, 60))
            b.apply_jacobian(x)
            ops[1].rotate_rotor(2.0, 1.0)  # member now holds no linearization at its angle
            with pytest.raises(binding.MnsError) as e1:
                b.apply_jacobian(x)
            assert e1.value.code == binding.MNS_ERR_NOT_LINEARIZED
            _, rc, _ = b.solve(x, check=False, precond="f64", restart=10, maxit=5)
            assert rc == binding.MNS_ERR_NOT_LINEARIZED
            ops[1].set_linearization(_dev(inputs.uniform(n, 51)))
            b.apply_jacobian(x)
            torch.cuda.synchronize()
    finally:
        for op in ops:
            op.close()


def test_stream_bandwidth_measurement():
    """mns_stream_bandwidth: the read-dominated stream rate used as the
    practical HBM ceiling is positive and below the HBM peak, and bad sizes
    or ratios are refused before any launch."""
    gbs = binding.stream_bandwidth(1 << 28, 6, 3)
    print(f"stream kernel: {gbs:.0f} GB/s")
    assert 100.0 < gbs < 8000.0
    for rb, ratio in ((1 << 10, 6), (1 << 28, 0), (1 << 28, 65)):
        with pytest.raises(binding.MnsError) as e:
            binding.stream_bandwidth(rb, ratio, 1)
        assert e.value.code == binding.MNS_ERR_INVALID_ARG
