"""Allocation-free Jacobian application (mns_apply_jacobian_noalloc) against
mns_apply_jacobian through the C-ABI: the same kernels on the same inputs,
with the local results in the library's scratch array instead of the handle's
buffers, so the products agree bit for bit.  Two calls in a row, the second on
a smaller mesh (the array keeps the first call's contents), in FP64 and FP32,
2D and 3D, every launch mode; a mesh whose local results exceed the array is
refused with UNSUPPORTED."""
import numpy as np
import pytest

from paper_2608_27423_amd import binding, inputs
from tests.helpers import small_mesh

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _pair(mesh, seed, theta, fused, dtype):
    n = inputs.n_dofs(mesh)
    state = torch.from_numpy(inputs.uniform(n, seed)).cuda()
    x = torch.from_numpy(inputs.uniform(n, seed + 1)).cuda().to(dtype)
    with binding.Operator(mesh) as op:
        op.set_kernel_config(fused_launch=fused)
        op.rotate_rotor(theta, 0.9)
        op.set_linearization(state)
        ref = op.apply_jacobian(x)
        y = torch.full_like(x, float("nan"))
        op.apply_jacobian_noalloc(x, y)
        torch.cuda.synchronize()
        return ref.cpu().numpy(), y.cpu().numpy()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("fused", [0, 1, 2])
@pytest.mark.parametrize("dim", [2, 3])
def test_noalloc_equals_apply_two_calls(dim, fused, dtype):
    dt = torch.float64 if dtype == "f64" else torch.float32
    big = small_mesh(dim, 2, n_theta=32, n_r_rotor=3, n_r_stator=4, n_z=6)
    small = small_mesh(dim, 2, n_theta=16, n_r_rotor=2, n_r_stator=2, n_z=2)
    for i, (mesh, theta) in enumerate(((big, 0.61), (small, 2.2))):
        ref, y = _pair(mesh, 70 + 10 * i, theta, fused, dt)
        print(f"dim={dim} fused={fused} {dtype} call {i}: n={ref.size} equal={np.array_equal(ref, y)}")
        assert np.array_equal(ref, y)


def test_noalloc_workload_size_and_refusal():
    # the 3D Q2 64 x 8 x 32 per domain workload fits the array
    name = "annulus3d_q2_64x8x32"
    mesh = inputs.mesh(name)
    state = torch.from_numpy(inputs.state_for(name)).cuda()
    x = torch.from_numpy(inputs.vector_for(name)).cuda()
    with binding.Operator(mesh) as op:
        op.rotate_rotor(inputs.rotor_angle(name), mesh["omega"])
        op.set_linearization(state)
        ref = op.apply_jacobian(x)
        y = torch.empty_like(x)
        op.apply_jacobian_noalloc(x, y)
        torch.cuda.synchronize()
        assert torch.equal(ref, y)
    # 20 % more layers: more local results than the array holds
    too_big = dict(mesh, n_z=40)
    with binding.Operator(too_big) as op:
        op.rotate_rotor(0.3, 1.0)
        op.set_linearization(torch.zeros(op.n_dofs, dtype=torch.float64, device="cuda"))
        xx = torch.zeros(op.n_dofs, dtype=torch.float64, device="cuda")
        with pytest.raises(binding.MnsError) as e:
            op.apply_jacobian_noalloc(xx, torch.empty_like(xx))
        assert e.value.code == binding.MNS_ERR_UNSUPPORTED
        assert "scratch" in str(e.value)
