"""Linearization source C (tau and tau R stored per point; the advection
velocity a = u - w and grad u evaluated from the state inside the quad volume
kernel, Sec. 2.3) against the oracle and against source B, through the C-ABI.

FP64 (3D degree 2) to the parity bar 1e-12; FP32 (3D degrees 2 and 3) to the
FP32 bound.  Cases: every launch mode, steady and BDF2 (history and force in
tau R), Newton and Picard, rotor angles generic and aligned, spinning rotor
(mesh velocity in a), ring lengths with and without the strip layout; the
switch back to source B; where source C does not exist the setting is
ignored; the autotuner reports a valid choice."""
import math

import numpy as np
import pytest
import torch

import oracle
from helpers import oracle_cfg, relmax, small_mesh
from paper_2608_27423_amd import binding, inputs

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 5e-5


def _dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def _applies(op, x):
    y64 = op.apply_jacobian(_dev(x)).cpu().numpy()
    y32 = op.apply_jacobian(_dev(x, torch.float32)).double().cpu().numpy()
    return y64, y32


@pytest.mark.parametrize("k", [2, 3])
@pytest.mark.parametrize("n_theta", [5, 16])
@pytest.mark.parametrize("steady,kind", [(1, "newton"), (0, "newton"), (1, "picard"), (0, "picard")])
@pytest.mark.parametrize("fused", [1, 0, 2])
def test_source_c_matches_oracle(k, n_theta, steady, kind, fused):
    mesh = small_mesh(3, k, n_theta=n_theta, steady=steady, dt=0.05)
    n = inputs.n_dofs(mesh)
    g = np.random.default_rng(500 + 10 * k + n_theta + 2 * steady)
    state, x, hist, force = (g.uniform(-1, 1, n) for _ in range(4))
    hist = None if steady else hist
    dth = 2 * math.pi / n_theta
    for theta, omega in ((2.345, 0.8), (3 * dth, -1.3)):
        cfg = oracle_cfg(mesh, theta, omega)
        yo = oracle.apply_jacobian(dict(cfg, picard=int(kind == "picard")), state, x, hist=hist, force=force)
        with binding.Operator(mesh) as op:
            op.rotate_rotor(theta, omega)
            op.set_linearization(_dev(state), None if hist is None else _dev(hist), _dev(force), kind=kind)
            op.set_kernel_config(fused_launch=fused, volume_layout=1, lin_source_f64=0, lin_source_f32=0)
            b64, b32 = _applies(op, x)
            op.set_kernel_config(lin_source_f64=1, lin_source_f32=1)
            assert op.get_kernel_config()["lin_source_f64"] == 1
            c64, c32 = _applies(op, x)
        e = dict(b64=relmax(b64, yo), c64=relmax(c64, yo), b32=relmax(b32, yo), c32=relmax(c32, yo),
                 bc64=relmax(c64, b64))
        print(f"k={k} nt={n_theta} steady={steady} {kind} fused={fused} theta={theta:.3f}: "
              + " ".join(f"{a} {v:.2e}" for a, v in e.items()))
        assert e["b64"] <= TOL64 and e["c64"] <= TOL64
        assert e["b32"] <= TOL32 and e["c32"] <= TOL32


def test_source_c_fp32_differs_from_b_only_by_rounding():
    """FP32 sources B and C round differently (C evaluates a and grad u from
    the FP32 state, B rounds the FP64 values), so they differ, but only at
    FP32 rounding level; in FP64 (degree 2) they agree to 1e-13."""
    mesh = small_mesh(3, 2, n_theta=16, n_r_rotor=2, n_r_stator=2, n_z=4)
    n = inputs.n_dofs(mesh)
    g = np.random.default_rng(77)
    state, x = g.uniform(-1, 1, n), g.uniform(-1, 1, n)
    with binding.Operator(mesh) as op:
        op.rotate_rotor(0.77, 1.0)
        op.set_linearization(_dev(state))
        op.set_kernel_config(fused_launch=1, lin_source_f64=0, lin_source_f32=0)
        b64, b32 = _applies(op, x)
        op.set_kernel_config(lin_source_f64=1, lin_source_f32=1)
        c64, c32 = _applies(op, x)
        op.set_kernel_config(lin_source_f64=0, lin_source_f32=0)
        b64_again, b32_again = _applies(op, x)
    print(f"C vs B: fp64 {relmax(c64, b64):.2e}, fp32 {relmax(c32, b32):.2e}")
    assert relmax(c64, b64) <= 1e-13
    assert 0 < relmax(c32, b32) <= 1e-5
    assert np.array_equal(b64, b64_again) and np.array_equal(b32, b32_again)


@pytest.mark.parametrize("dim,k,layout", [(2, 2, 1), (3, 4, 1), (3, 2, 0)])
def test_source_c_setting_ignored_where_absent(dim, k, layout):
    """2D, degree 4 and the LDS-plane layout have no source C: the setting is
    accepted and the product is source B's, bit for bit."""
    mesh = small_mesh(dim, k)
    n = inputs.n_dofs(mesh)
    g = np.random.default_rng(9 + k)
    state, x = g.uniform(-1, 1, n), g.uniform(-1, 1, n)
    with binding.Operator(mesh) as op:
        op.rotate_rotor(1.3, 0.5)
        op.set_linearization(_dev(state))
        op.set_kernel_config(fused_launch=1, volume_layout=layout, lin_source_f64=0, lin_source_f32=0)
        b64, b32 = _applies(op, x)
        op.set_kernel_config(lin_source_f64=1, lin_source_f32=1)
        c64, c32 = _applies(op, x)
    assert np.array_equal(b64, c64) and np.array_equal(b32, c32)


def test_source_c_invalid_and_autotune():
    mesh = small_mesh(3, 2, n_theta=16)
    n = inputs.n_dofs(mesh)
    with binding.Operator(mesh) as op:
        op.rotate_rotor(0.4, 1.0)
        op.set_linearization(_dev(inputs.uniform(n, 3)))
        with pytest.raises(binding.MnsError) as e:
            op.set_kernel_config(lin_source_f64=2)
        assert e.value.code == binding.MNS_ERR_INVALID_ARG
        with pytest.raises(TypeError):
            op.set_kernel_config(lin_source=1)
        chosen = op.autotune_kernel_config(reps=3)
        print("autotune:", chosen)
        assert chosen == op.get_kernel_config()
        assert chosen["lin_source_f64"] in (0, 1) and chosen["lin_source_f32"] in (0, 1)
        x = _dev(inputs.uniform(n, 4))
        y = op.apply_jacobian(x).cpu().numpy()
        yo = oracle.apply_jacobian(oracle_cfg(mesh, 0.4, 1.0), inputs.uniform(n, 3), x.cpu().numpy())
        assert relmax(y, yo) <= TOL64
