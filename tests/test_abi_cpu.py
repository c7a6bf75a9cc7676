"""Host-side checks of the C-ABI library that need no GPU: it loads, exports
every entry point declared in include/mortarns.h, and rejects invalid meshes
before touching the device."""
import ctypes
import os
import re

import pytest

from paper_2608_27423_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "mortarns.h")).read()
    return sorted(set(re.findall(r"\b(mns_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_binding_names():
    assert _declared() == sorted(binding.EXPORTED)


def test_library_exports_every_declared_symbol():
    L = binding.lib()
    for name in _declared():
        assert hasattr(L, name), name


@pytest.mark.parametrize("bad", [
    dict(dim=4), dict(degree=1), dict(degree=9), dict(r_in=0.6), dict(r_out=0.4), dict(n_theta=2),
    dict(n_r_rotor=0), dict(nu=0.0), dict(penalty_F=-1.0), dict(penalty_rule=3), dict(steady=0, dt=0.0),
    dict(dim=3, n_z=0), dict(dim=3, height=-1.0),
])
def test_invalid_mesh_rejected(bad):
    mesh = dict(dim=2, degree=2, r_in=0.25, r_if=0.5, r_out=1.0, height=1.0, n_theta=8, n_r_rotor=2, n_r_stator=2,
                n_z=2, nu=0.01, penalty_F=1.0, penalty_rule=0, steady=1, dt=1.0)
    mesh.update(bad)
    desc = binding.mesh_desc(mesh)
    L = binding.lib()
    h = ctypes.c_void_p()
    rc = L.mns_setup_mesh(ctypes.byref(desc), None, ctypes.byref(h))
    try:
        assert rc in (binding.MNS_ERR_INVALID_ARG, binding.MNS_ERR_UNSUPPORTED)
        assert L.mns_last_error(h).decode() != ""
    finally:
        L.mns_destroy(h)


def test_null_arguments():
    L = binding.lib()
    assert L.mns_setup_mesh(None, None, None) == binding.MNS_ERR_INVALID_ARG
    assert L.mns_rotate_rotor(None, 0.0, 0.0, None) == binding.MNS_ERR_INVALID_ARG
    assert L.mns_apply_jacobian(None, 0, None, None, None) == binding.MNS_ERR_INVALID_ARG
    assert L.mns_last_error(None) == b"null handle"


def test_solve_options_are_checked_by_name():
    """Options reach the library only through the struct's own fields: an
    unknown name is an error (a plain setattr would be silently ignored), and
    the string forms map to the header's constants."""
    o = binding.Operator.default_solve_opts()
    assert o.cheb_lambda_factor == pytest.approx(1.05)
    with pytest.raises(TypeError):
        binding._set_fields(o, {"cheb_degre": 8})
    binding._set_fields(o, {"precond": "mg64", "mg_coarse_linearization": "picard", "cheb_degree": 9})
    assert (o.precond, o.mg_coarse_linearization, o.cheb_degree) == (
        binding.MNS_PRECOND_MG64, binding.MNS_LIN_PICARD, 9)


def test_bench_refuses_more_than_one_gpu():
    """bench.py --gpus N with N > 1 exits with a message instead of running."""
    import json
    import subprocess
    import sys

    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2
    msg = json.loads(p.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]


def test_bench_roofline_bookkeeping():
    """The bench's roofline bookkeeping on the workloads: algorithmic bytes per
    launch (src + dst once, 16 FP64 values per Gauss point; source C: 4 values
    per point and the state's velocity) and the name of the
    launch its volume timer brackets under the automatic launch mode (fused
    below 262,144 cells, the volume kernel beside a second-stream mortar
    launch from there on; degree-2 FP64 fused launch in its LDS-staged form)."""
    import sys

    sys.path.insert(0, ROOT)
    import bench
    from paper_2608_27423_amd import inputs

    c2 = inputs.mesh("annulus3d_q2_64x8x32")
    b, cells = bench.algorithmic_bytes_volume(c2, inputs.n_dofs(c2), 8)
    assert (b, cells) == (131350528, 32768)
    assert bench.dominant_kernel(c2, -1, 1) == "mns::k_jacobian_fused_quad_lds<3, false>"
    assert bench.dominant_kernel(c2, -1, 1, "double", 1) == "mns::k_jacobian_fused_quad_lds<3, true>"
    assert bench.dominant_kernel(c2, -1, 1, "float") == "mns::k_jacobian_fused_quad<float, 3, false>"
    assert bench.dominant_kernel(c2, 0, 1) == "mns::k_jacobian_volume_quad<double, 3, false>"
    assert bench.dominant_kernel(c2, -1, 0) == "mns::k_jacobian_fused<double, 3, 3>"
    # source C: src + dst + the state's velocity once, 4 values per Gauss point
    n2 = inputs.n_dofs(c2)
    assert bench.algorithmic_bytes_volume(c2, n2, 8, 1)[0] == (2.75 * n2 + 4 * 27 * 32768) * 8
    c5 = inputs.mesh("annulus3d_q2_256x32x128")
    assert bench.algorithmic_bytes_volume(c5, inputs.n_dofs(c5), 8)[0] == 8342536192
    assert bench.dominant_kernel(c5, -1, 1) == "mns::k_jacobian_volume_quad<double, 3, false>"
    c3 = inputs.mesh("annulus3d_q3_64x16x32")
    assert bench.dominant_kernel(c3, -1, 1) == "mns::k_jacobian_fused_quad<double, 4, false>"
    # degree 3 has source C in FP32 only
    assert bench.dominant_kernel(c3, -1, 1, "double", 1) == "mns::k_jacobian_fused_quad<double, 4, false>"
    assert bench.dominant_kernel(c3, -1, 1, "float", 1) == "mns::k_jacobian_fused_quad<float, 4, true>"
    c1 = inputs.mesh("annulus2d_q2_32x4")
    assert bench.dominant_kernel(c1, -1, 1) == "mns::k_jacobian_fused<double, 2, 3>"


def test_bench_traffic_summary_parsing(tmp_path, monkeypatch):
    """bench.measured_traffic reads the per-application and per-launch HBM
    bytes of a counter summary whose keys hold kernel names with '::', and
    returns nothing once the kernel source digest no longer matches."""
    import sys

    sys.path.insert(0, ROOT)
    import bench

    prof = tmp_path / "profiles"
    prof.mkdir()
    digest = bench.kernel_source_digest()
    (prof / "traffic_w.txt").write_text(
        "# comment: with a colon\n"
        f"kernel_source_sha256: {digest}\n"
        "bytes_per_launch mns::k_a<double, 3, false>: 1000\n"
        "read_write_per_launch mns::k_a<double, 3, false>: 600 400\n"
        "vmult_bytes_per_call: 1500\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_digest", lambda: digest)
    assert bench.measured_traffic("w", "mns::k_a<double, 3, false>") == (1500.0, 1000.0)
    assert bench.measured_traffic("w", "mns::k_b") == (1500.0, None)
    assert bench.measured_traffic("missing", "mns::k_a") == (None, None)
    monkeypatch.setattr(bench, "kernel_source_digest", lambda: "other")
    assert bench.measured_traffic("w", "mns::k_a<double, 3, false>") == (None, None)
