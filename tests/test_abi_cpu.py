"""The C ABI without a GPU: the library loads, exports every entry point the
header declares, validates arguments before touching HIP, and its host-side
geometry (Sec. II.B-II.C) agrees with the oracle."""
import os
import re

import numpy as np
import pytest

from oracle import pulse as opulse
from paper_2010_00409_amd import tfocus as tf
from synthetic import configs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "tfocus.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tf_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_entry_point():
    lib = tf.load()
    names = header_functions()
    assert len(names) >= 17
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(tf.exported_names())


def test_version_and_supported_lengths():
    assert tf.tf_version().startswith("tfocus")
    for n in (8, 16, 24, 64, 96, 192, 512, 768, 1024, 40, 80, 640, 56, 112, 896):
        assert tf.tf_supported_length(n)
    for n in (4, 10, 100, 2048, 72, 88, 1536, 1120):
        assert not tf.tf_supported_length(n)


@pytest.mark.parametrize("grid, prec, status", [
    (dict(configs.cube_grid(64, 0.1), nx=63), "f32", tf.TF_EINVAL),
    (dict(configs.cube_grid(64, 0.1), nx=100), "f32", tf.TF_EUNSUPPORTED),
    (dict(configs.cube_grid(64, 0.1), ny=2048), "f32", tf.TF_EUNSUPPORTED),
    (dict(configs.cube_grid(64, 0.1), dx=0.0), "f32", tf.TF_EINVAL),
    (dict(configs.cube_grid(64, 0.1), dz=float("nan")), "f64", tf.TF_EINVAL),
    (configs.cube_grid(64, 0.1), 7, tf.TF_EINVAL),
])
def test_create_rejects_bad_descriptors(grid, prec, status):
    with pytest.raises(tf.TfError) as ei:
        tf.tf_create(grid, prec)
    assert ei.value.status == status
    assert tf.tf_last_error()


def test_device_byte_cap_gives_enomem_before_any_hip_call(monkeypatch):
    monkeypatch.setenv("TFOCUS_MAX_DEVICE_BYTES", "1000000")
    with pytest.raises(tf.TfError) as ei:
        tf.tf_create(configs.cube_grid(64, 0.1), "f32")
    assert ei.value.status == tf.TF_ENOMEM


@pytest.mark.parametrize("bad, status", [
    (dict(wavelength=0.0), tf.TF_EINVAL),
    (dict(R0=0.5, L=2.0), tf.TF_EINVAL),
    (dict(theta=0.0, f_number=0.0), tf.TF_EINVAL),
    (dict(envelope="spectral", nfreq=0), tf.TF_EINVAL),
    (dict(polarization="radial", ellipticity=0.5), tf.TF_EINVAL),
])
def test_pulse_validation(bad, status):
    with pytest.raises(tf.TfError) as ei:
        tf.tf_pulse_geometry(configs.pulse(**bad))
    assert ei.value.status == status


def test_null_pointers_are_rejected():
    lib = tf.load()
    assert lib.tf_create(None, 0, None, None) == tf.TF_EINVAL
    assert lib.tf_advance(None, 1, 0.1) == tf.TF_EINVAL
    assert lib.tf_read_focal(None, None, None, 0) == tf.TF_EINVAL
    assert lib.tf_destroy(None) == tf.TF_OK


@pytest.mark.parametrize("kw", [
    dict(f_number=0.3), dict(f_number=0.5, eps=0.2), dict(theta=0.9, R0=6.0, L=10.0),
    dict(transverse="gauss", f_number=1.0), dict(transverse="gauss", f_number=0.25, R0=20.0, L=24.0),
])
def test_pulse_geometry_matches_oracle(kw):
    p = configs.pulse(**kw)
    got = tf.tf_pulse_geometry(p)
    ref = opulse.geometry(p)
    for k in ("theta", "R_min", "R_max", "L", "D_min", "alpha_max"):
        assert got[k] == pytest.approx(ref[k], rel=1e-15, abs=1e-15), k
    assert got["A"] == pytest.approx(ref["A"], rel=1e-12)


@pytest.mark.parametrize("n, d", [((56, 64, 64), 0.125), ((256, 256, 256), 0.125),
                                  ((512, 512, 512), 1 / 12), ((42, 30, 18), 0.3)])
def test_layer_grid_matches_oracle(n, d):
    for p in (configs.c2()["pulse"], configs.c3()["pulse"], configs.pulse()):
        got = tf.tf_layer_grid(p, n, (d, d, d))
        ref = opulse.layer_grid(p, n, (d, d, d))
        assert got == ref


def test_surrogate_arguments_are_validated_before_any_hip_call():
    import ctypes
    lib = tf.load()
    h = ctypes.c_void_p()
    assert lib.tf_fno_create(0, 0, 1, None, ctypes.byref(h)) == tf.TF_EINVAL
    assert lib.tf_fno_create(129, 0, 1, None, ctypes.byref(h)) == tf.TF_EINVAL
    assert lib.tf_fno_create(4, 0, 3, None, ctypes.byref(h)) == tf.TF_EINVAL
    assert lib.tf_fno_create(4, 0, 1, None, None) == tf.TF_EINVAL
    assert [lib.tf_fno_param_count(k) for k in (0, 1, 2, 3, 4)] == \
        [-1, lib.tf_fno_param_count(1), lib.tf_fno_param_count(1) + 774, -1, lib.tf_fno_param_count(1) + 2322]
    assert lib.tf_fno_forward(None, None, None, 1, None) == tf.TF_EINVAL
    assert lib.tf_fno_infer(None, None, None, 1, None) == tf.TF_EINVAL
    assert lib.tf_fno_train_step(None, None, None, None, 1, 1e-3, None) == tf.TF_EINVAL
    assert lib.tf_fno_destroy(None) == tf.TF_OK
    w = (ctypes.c_double * 4)()
    assert lib.tf_fno_phasor_weights(ctypes.byref(tf.pulse_struct(configs.pulse())), 3, w) == tf.TF_EINVAL
    assert lib.tf_fno_phasor_weights(None, 2, w) == tf.TF_EINVAL


def test_surrogate_head_weights_of_a_plain_pulse():
    """Linear polarisation along y, no ellipticity, CEP 0, cos^2 envelope
    (s = -1, gnorm 1): weights (1, 0, 0, 0) for four basis fields."""
    import numpy as np
    w = tf.tf_fno_phasor_weights(configs.pulse(cep=0.0, pol_angle=0.0, ellipticity=0.0), 4)
    assert np.allclose(w, [1, 0, 0, 0], atol=1e-15)
    w2 = tf.tf_fno_phasor_weights(configs.pulse(cep=0.5 * np.pi, pol_angle=0.5 * np.pi), 4)
    # z = exp(-i pi/2) = -i, b = 1: Re(z b) = 0, -Im(z b) = 1
    assert np.allclose(w2, [0, 0, 0, 1], atol=1e-15)


def test_fast_z_kernel_needs_its_strip_offsets_to_fit_32_bits(monkeypatch):
    """The fast z kernel addresses a strip with 32-bit byte offsets spanning
    (nz - 1) row blocks of 6 nx/2 complex values: an unblocked 768 x 512 x 512
    spectrum (4.8 GB) must fall to the generic kernels, blocked rows and the
    unblocked 512^3 (3.2 GB) keep the fast ones.  Decided on the host."""
    monkeypatch.delenv("TFOCUS_GENERIC_KERNELS", raising=False)
    monkeypatch.delenv("TFOCUS_ZVARIANT", raising=False)
    wide = dict(configs.cube_grid(512, 0.1), nx=768)
    for grid, rb, fast in ((wide, "512", False), (wide, "8", True),
                           (configs.cube_grid(512, 0.1), "512", True)):
        monkeypatch.setenv("TFOCUS_ROW_BLOCK", rb)
        got_rb, got_fast, _, _ = tf.tf_kernel_plan(grid, "f32")
        assert got_rb == int(rb) and got_fast == fast, (grid["nx"], rb)
    # the arithmetic behind the decision: last strip offset of the wide grid
    rowb = 6 * (768 // 2) * 8
    assert (511 * 512 + 1) * rowb > 2 ** 32 >= (511 * 8 + 1) * rowb
    with pytest.raises(tf.TfError):
        tf.tf_kernel_plan(dict(wide, nx=100), "f32")


def test_plan_file_lines_with_and_without_the_y_strip_width(tmp_path, monkeypatch):
    """Plan lines carry the y strip width before the timing; older lines
    without it keep 64-column strips; a bad width drops the line; the
    TFOCUS_YSTRIP override takes 64 or 32.  Host only (the plan lookup runs
    before any HIP call; without a device the architecture reads 'unknown')."""
    for v in ("TFOCUS_ROW_BLOCK", "TFOCUS_GENERIC_KERNELS", "TFOCUS_ZVARIANT", "TFOCUS_YSTRIP"):
        monkeypatch.delenv(v, raising=False)
    plan = tmp_path / "plans.txt"
    plan.write_text("# comment\n"
                    "unknown f32 128 128 128 128 1 6 32 0.1\n"
                    "unknown f32 192 192 192 8 1 5 0.3\n"
                    "unknown f32 256 256 256 256 1 4 48 0.7\n")
    old = os.environ.get("TFOCUS_PLAN_FILE") or tf.DEFAULT_PLANS
    tf.tf_set_plan_file(str(plan))
    try:
        assert tf.tf_kernel_plan(configs.cube_grid(128, 0.1), "f32") == (128, True, 6, 32)
        assert tf.tf_kernel_plan(configs.cube_grid(192, 0.1), "f32") == (8, True, 5, 64)
        assert tf.tf_kernel_plan(configs.cube_grid(256, 0.1), "f32") == (8, True, 0, 64)
        monkeypatch.setenv("TFOCUS_YSTRIP", "32")
        assert tf.tf_kernel_plan(configs.cube_grid(192, 0.1), "f32")[3] == 32
        monkeypatch.setenv("TFOCUS_YSTRIP", "48")
        assert tf.tf_kernel_plan(configs.cube_grid(192, 0.1), "f32")[3] == 64
    finally:
        tf.tf_set_plan_file(old)


def test_phase_bumps_are_validated_before_any_hip_call():
    p = configs.pulse()
    assert tf.tf_pulse_geometry(dict(p, bumps=[(0.0, 0.1, 0.5, 0.2)]))["theta"] > 0
    for bad in ([(0.0, 0.1, 0.5, 0.0)], [(float("nan"), 0.1, 0.5, 0.2)]):
        with pytest.raises(tf.TfError) as ei:
            tf.tf_pulse_geometry(dict(p, bumps=bad))
        assert ei.value.status == tf.TF_EINVAL
    s = tf.pulse_struct(p)
    s.nbumps = 3                                   # count without a table
    with pytest.raises(tf.TfError):
        tf.tf_pulse_geometry(s)
