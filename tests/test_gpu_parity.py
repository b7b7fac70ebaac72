"""GPU parity: the HIP path through the C ABI against the float64 oracle on
the same seeded inputs.  Tolerances (relative L2 over all six components):
float64 <= 1e-12, float32 <= 1e-5 per step."""
import math

import numpy as np
import pytest

from oracle import mapping, psatd, pulse
from paper_2010_00409_amd import tfocus as tf
from synthetic import configs, planewaves

pytestmark = pytest.mark.gpu

F64_TOL = 1e-12
F32_TOL = 1e-5


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def spacing(g):
    return (g["dz"], g["dy"], g["dx"])


def run_gpu(grid, prec, state, nsteps, dt, t0=0.0):
    dtype = np.float64 if prec == "f64" else np.float32
    with tf.Solver(grid, prec) as s:
        s.set_fields(np.ascontiguousarray(state, dtype=dtype), t0)
        s.advance(nsteps, dt)
        out = np.empty(s.shape, dtype=dtype)
        s.get_fields(out)
        return out, s.t


def transverse_state(seed, shape, d):
    g = dict(nx=shape[2], ny=shape[1], nz=shape[0], dx=d, dy=d, dz=d, x_min=0.0, y_min=0.0, z_min=0.0)
    E, B = planewaves.random_fields(seed, shape)
    E, B = psatd.step_fft(E, B, spacing(g), 0.0, project_b_first=True)
    return g, np.concatenate([E, B])


def test_roundtrip_is_bitwise():
    g = configs.cube_grid(32, 0.25)
    for prec, dt in (("f64", np.float64), ("f32", np.float32)):
        x = np.random.default_rng(0).standard_normal((6, 32, 32, 32)).astype(dt)
        out, t = run_gpu(g, prec, x, 0, 0.1, t0=1.5)
        assert np.array_equal(out, x) and t == 1.5


def test_C1_planewaves_f64_64_steps_match_oracle_and_closed_form():
    c = configs.c1()
    g = c["grid"]
    modes = planewaves.draw(c["planewave_seed"], nmodes=16, mmax=31)
    E, B = planewaves.fields(modes, g)
    out, t = run_gpu(g, "f64", np.concatenate([E, B]), c["steps"], c["dt"])
    Eo, Bo = psatd.step_fft(E, B, spacing(g), c["dt"], nsteps=c["steps"])
    ref = np.concatenate([Eo, Bo])
    assert rel(out, ref) <= F64_TOL
    assert t == 0.0 + c["steps"] * c["dt"]


def test_C1_pulse_f64_init_and_64_steps_match_oracle():
    c = configs.c1()
    g = c["grid"]
    with tf.Solver(g, "f64") as s:
        info = s.set_pulse(c["pulse"])
        init = np.empty(s.shape)
        s.get_fields(init)
        s.advance(c["steps"], c["dt"])
        out = np.empty(s.shape)
        s.get_fields(out)
    E, B = pulse.init_fields(c["pulse"], g)
    ref0 = np.concatenate([E, B])
    assert rel(init, ref0) <= F64_TOL
    assert np.abs(init).max() > 0.01
    Eo, Bo = psatd.step_fft(E, B, spacing(g), c["dt"], nsteps=c["steps"], project_b_first=True)
    assert rel(out, np.concatenate([Eo, Bo])) <= F64_TOL
    assert info["R_min"] == pulse.geometry(c["pulse"])["R_min"]


SHAPES = [(8, 8, 8), (16, 24, 32), (8, 8, 1024), (8, 1024, 8), (1024, 8, 8), (24, 48, 96),
          (12 * 2, 16, 768), (16, 384, 8), (192, 8, 16), (64, 64, 64), (32, 128, 256), (16, 512, 16),
          (512, 16, 8), (16, 64, 32), (8, 256, 96)]     # the last two: 256-byte y strips


@pytest.mark.parametrize("shape", SHAPES, ids=[f"{s[2]}x{s[1]}x{s[0]}" for s in SHAPES])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_one_step_every_axis_length(shape, prec):
    """shape = (nz, ny, nx); one step of a random transverse field (plus a
    second with the B projection) against the oracle."""
    g, st = transverse_state(sum(shape), shape, 0.37)
    dtype = np.float64 if prec == "f64" else np.float32
    st = st.astype(dtype).astype(np.float64)
    out, _ = run_gpu(g, prec, st, 1, 0.61)
    Eo, Bo = psatd.step_fft(st[:3], st[3:], spacing(g), 0.61)
    assert rel(out.astype(np.float64), np.concatenate([Eo, Bo])) <= (F64_TOL if prec == "f64" else F32_TOL)


def test_f32_step_random_longitudinal_input_and_b_projection():
    """Unstructured input: the step must also remove longitudinal E (Eq. (3))
    and, on the first step after a pulse, longitudinal B."""
    shape = (32, 48, 64)
    g = dict(nx=64, ny=48, nz=32, dx=0.3, dy=0.25, dz=0.2, x_min=-1.0, y_min=2.0, z_min=0.5)
    x = np.random.default_rng(5).standard_normal((6,) + shape).astype(np.float32)
    out, _ = run_gpu(g, "f32", x, 1, 0.45)
    Eo, Bo = psatd.step_fft(x[:3].astype(np.float64), x[3:].astype(np.float64), spacing(g), 0.45)
    assert rel(out.astype(np.float64), np.concatenate([Eo, Bo])) <= F32_TOL


@pytest.mark.parametrize("envelope, transverse, pol", [
    ("cos2", "flattop", "linear"), ("gauss", "gauss", "linear"), ("spectral", "flattop", "radial"),
    ("spectral", "gauss", "linear")])
def test_init_map_f64_matches_oracle(envelope, transverse, pol):
    p = configs.pulse(envelope=envelope, transverse=transverse, polarization=pol, R0=5.0, L=3.0,
                      f_number=0.6, ncycles=1.5, bandwidth=0.4, gdd=0.3, tod=0.05, cep=0.8,
                      ellipticity=0.0 if pol == "radial" else 0.4, pol_angle=0.3, nfreq=96)
    g = pulse.layer_grid(p, (24, 64, 48), (0.2, 0.21, 0.22))     # D = 4.8 < D_min: overlap
    with tf.Solver(g, "f64") as s:
        info = s.set_pulse(p)
        out = np.empty(s.shape)
        s.get_fields(out)
    E, B = pulse.init_fields(p, g)
    ref = np.concatenate([E, B])
    assert np.abs(ref).max() > 0.01
    assert rel(out, ref) <= F64_TOL
    assert info["overlap"] == (info["D"] < info["D_min"])


def test_readout_matches_oracle_bitwise_f64():
    p = configs.pulse(envelope="cos2", R0=4.0, L=2.0, theta=1.0)
    g = pulse.layer_grid(p, (48, 64, 64), (0.125, 0.125, 0.125))
    geo = pulse.geometry(p)
    win = dict(wx=40, wy=36, wz=30, cx=0.3, cy=-0.2, cz=0.1)
    for T in (0.0, 1.7, 4.0, 6.5):
        with tf.Solver(g, "f64") as s:
            s.set_pulse(p)
            s.advance(1, T)
            full = np.empty(s.shape)
            s.get_fields(full)
            out = np.empty((6, 30, 36, 40))
            s.read_focal(win, out)
            tt = s.t
        ref = mapping.readout(full, g, win, tt, geo["R_min"], geo["R_max"])
        assert np.array_equal(out, ref)


def test_transverse_replication_init_and_wrapped_window_match_oracle():
    """Duplication along y and z (Sec. II.C closing remarks), float64: the
    replicated init of a small transverse box and a focal window wider than
    the box (wrapping in y and z) against the oracle."""
    p = configs.pulse(envelope="spectral", bandwidth=0.4, R0=4.0, L=2.0, theta=0.8, eps=0.1, nfreq=64)
    d = 0.25
    g = dict(pulse.layer_grid(p, (16, 16, 24), (d, d, d)), replicate_yz=1)
    with tf.Solver(g, "f64") as s:
        s.set_pulse(p)
        st = np.empty(s.shape)
        s.get_fields(st)
        win = dict(wx=8, wy=24, wz=40, cx=0.0, cy=0.3, cz=-0.2)
        w = np.empty((6, 40, 24, 8))
        s.read_focal(win, w)
    E, B = pulse.init_fields(p, g)
    ref = np.concatenate([E, B])
    assert np.abs(ref).max() > 0.1
    assert rel(st, ref) <= F64_TOL
    geo = pulse.geometry(p)
    assert np.array_equal(w, mapping.readout(st, g, win, 0.0, geo["R_min"], geo["R_max"]))


@pytest.mark.parametrize("envelope", ["cos2", "spectral"])
def test_phase_perturbed_init_matches_oracle(envelope):
    """Wavefront phase bumps (Sec. III.B.3) in the init, float64, against the
    oracle: 44 bumps of width 0.3 theta over the aperture."""
    from paper_2010_00409_amd import verify
    p = configs.pulse(envelope=envelope, R0=4.0, L=2.0, f_number=1.0, eps=0.1, nfreq=64, cep=0.4)
    th = pulse.geometry(p)["theta"]
    p = dict(p, bumps=verify.phase_bumps(th, 0.8, np.random.default_rng(5)))
    g = pulse.layer_grid(p, (24, 48, 48), (0.2, 0.2, 0.2))
    with tf.Solver(g, "f64") as s:
        s.set_pulse(p)
        st = np.empty(s.shape)
        s.get_fields(st)
    E, B = pulse.init_fields(p, g)
    ref = np.concatenate([E, B])
    assert np.abs(ref).max() > 0.1
    assert rel(st, ref) <= F64_TOL
    E0, _ = pulse.init_fields(dict(p, bumps=None), g)
    assert rel(E0, E) > 0.1                         # the perturbation changes the field


def test_readout_rejects_window_outside_grid():
    g = configs.cube_grid(32, 0.25)
    with tf.Solver(g, "f32") as s:
        s.set_cutout(1.0, 2.0)
        with pytest.raises(tf.TfError) as ei:
            s.read_focal(dict(wx=8, wy=40, wz=8, cx=0, cy=0, cz=0), np.empty((6, 8, 40, 8), np.float32))
        assert ei.value.status == tf.TF_EINVAL
    with tf.Solver(g, "f32") as s:
        with pytest.raises(tf.TfError) as ei:
            s.read_focal(dict(wx=8, wy=8, wz=8, cx=0, cy=0, cz=0), np.empty((6, 8, 8, 8), np.float32))
        assert ei.value.status == tf.TF_ESTATE


def test_diagnostics_energy_and_divergence():
    g, st = transverse_state(21, (32, 32, 32), 0.3)
    with tf.Solver(g, "f64") as s:
        s.set_fields(st)
        e0, de, db = s.diagnostics()
        assert e0 == pytest.approx(psatd.energy(st[:3], st[3:]), rel=1e-13)
        assert de < 1e-13 and db < 1e-13
        s.advance(20, 0.77)
        e1, de1, db1 = s.diagnostics()
        assert e1 == pytest.approx(e0, rel=1e-12)
        assert de1 < 1e-12 and db1 < 1e-12
    x = np.random.default_rng(3).standard_normal((6, 32, 32, 32))
    with tf.Solver(g, "f64") as s:
        s.set_fields(x)
        _, de, db = s.diagnostics()
        rde, rdb = psatd.max_divergence(x[:3], x[3:], spacing(g))
        assert de == pytest.approx(rde, rel=1e-10) and db == pytest.approx(rdb, rel=1e-10)


def test_diagnostics_fused_into_the_last_step_f64():
    """tf_advance_diagnosed: the energy (Parseval on the updated spectrum)
    and the divergence ratios of the state after the steps, against the
    oracle's state and tf_diagnostics, for fields with longitudinal parts
    (B's survives the steps, E's is removed)."""
    g = dict(nx=24, ny=40, nz=32, dx=0.3, dy=0.25, dz=0.2, x_min=0.0, y_min=0.0, z_min=0.0)
    x = np.random.default_rng(8).standard_normal((6, 32, 40, 24))
    Eo, Bo = psatd.step_fft(x[:3], x[3:], spacing(g), 0.4, nsteps=3)
    with tf.Solver(g, "f64") as s:
        s.set_fields(x)
        en, de, db = s.advance_diagnosed(3, 0.4)
        out = np.empty(s.shape)
        s.get_fields(out)
        en2, de2, db2 = s.diagnostics()
        assert s.t == pytest.approx(1.2)
    assert rel(out, np.concatenate([Eo, Bo])) <= F64_TOL
    assert en == pytest.approx(psatd.energy(Eo, Bo), rel=1e-12)
    assert en == pytest.approx(en2, rel=1e-12)
    rde, rdb = psatd.max_divergence(Eo, Bo, spacing(g))
    assert rdb > 0.1 and db == pytest.approx(rdb, rel=1e-9) and db == pytest.approx(db2, rel=1e-9)
    assert de < 1e-13 and de2 < 1e-13 and rde < 1e-13
    with tf.Solver(g, "f64") as s:
        with pytest.raises(tf.TfError) as ei:
            s.advance_diagnosed(0, 0.4)
        assert ei.value.status == tf.TF_EINVAL


@pytest.mark.parametrize("shape", [(128, 128, 128), (512, 32, 64)])
def test_diagnostics_fused_into_the_last_step_f32(shape):
    """Float32 plans with fast kernels: the diagnosed step runs the generic z
    kernel; the state matches the oracle and the diagnostics those of
    tf_diagnostics on the same state and the oracle's energy."""
    g, st = transverse_state(31 + shape[0], shape, 0.27)
    st = st.astype(np.float32).astype(np.float64)
    Eo, Bo = psatd.step_fft(st[:3], st[3:], spacing(g), 0.35, nsteps=10)
    with tf.Solver(g, "f32") as s:
        s.set_fields(st.astype(np.float32))
        en, de, db = s.advance_diagnosed(10, 0.35)
        out = np.empty(s.shape, np.float32)
        s.get_fields(out)
        en2, de2, db2 = s.diagnostics()
    assert rel(out.astype(np.float64), np.concatenate([Eo, Bo])) <= 10 * F32_TOL
    assert en == pytest.approx(en2, rel=1e-5)
    assert en == pytest.approx(psatd.energy(Eo, Bo), rel=1e-5)
    assert de < 1e-5 and db < 1e-5 and de2 < 1e-5 and db2 < 1e-5


def test_reversibility_and_semigroup_on_gpu_f32():
    g, st = transverse_state(22, (64, 64, 64), 0.25)
    st = st.astype(np.float32)
    fwd, _ = run_gpu(g, "f32", st, 10, 0.3)
    back, _ = run_gpu(g, "f32", fwd, 10, -0.3)
    assert rel(back.astype(np.float64), st.astype(np.float64)) < 1e-5
    jump, _ = run_gpu(g, "f32", st, 1, 3.0)
    assert rel(fwd.astype(np.float64), jump.astype(np.float64)) < 1e-5


@pytest.mark.parametrize("zvariant", [3, 4, 5])
@pytest.mark.parametrize("dt", [1.0e4, -3.7e5])
def test_f32_huge_dt_step_matches_oracle(dt, zvariant, monkeypatch):
    """One float32 step with phases c |k| dt of 1e5-1e7 rad (Sec. II.A: the
    vacuum step is exact for any dt) against the oracle's float64 step: the
    float32 rotation's |k| and phase reduction must hold float64 accuracy."""
    monkeypatch.setenv("TFOCUS_ZVARIANT", str(zvariant))
    g, st = transverse_state(24, (64, 64, 64), 0.3)
    st = st.astype(np.float32).astype(np.float64)
    out, _ = run_gpu(g, "f32", st, 1, dt)
    Eo, Bo = psatd.step_fft(st[:3], st[3:], spacing(g), dt)
    assert rel(out.astype(np.float64), np.concatenate([Eo, Bo])) <= F32_TOL


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_graph_replayed_steps_equal_eager_steps_bitwise(prec):
    """tf_advance replays a captured graph of 8 steps and runs the remainder
    (and, after tf_set_pulse, the first step with the B projection) eagerly;
    with per-launch profiling every step is launched eagerly.  Both must give
    the same bits, across a re-capture for a new dt and a cached replay."""
    dtype = np.float64 if prec == "f64" else np.float32
    g, st = transverse_state(25, (32, 48, 64), 0.3)
    st = np.ascontiguousarray(st.astype(dtype))
    plan = [(21, 0.37), (16, -0.21), (9, 0.37), (3, 0.37)]
    outs = []
    for eager in (True, False):
        with tf.Solver(g, prec) as s:
            s.set_fields(st, 0.5)
            s.profile(eager)
            for n, dt in plan:
                s.advance(n, dt)
            out = np.empty(s.shape, dtype=dtype)
            s.get_fields(out)
            outs.append((out, s.t))
    assert np.array_equal(outs[0][0], outs[1][0])
    assert outs[0][1] == outs[1][1] == 0.5 + 21 * 0.37 + 16 * -0.21 + 9 * 0.37 + 3 * 0.37
    Eo, Bo = psatd.step_fft(st[:3].astype(np.float64), st[3:].astype(np.float64), spacing(g), 0.37, nsteps=21)
    Eo, Bo = psatd.step_fft(Eo, Bo, spacing(g), -0.21, nsteps=16)
    Eo, Bo = psatd.step_fft(Eo, Bo, spacing(g), 0.37, nsteps=12)
    tol = 1e-11 if prec == "f64" else 2 * F32_TOL
    assert rel(outs[1][0].astype(np.float64), np.concatenate([Eo, Bo])) <= tol


@pytest.mark.parametrize("zvariant", [0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11])
def test_every_z_variant_at_length_512(zvariant, monkeypatch):
    """512-point z columns (where variants 5 and 6 differ, residues are
    parked in LDS or held in registers, and variants 7 and 8 run one wave per
    mode) on a thin grid, two steps against the oracle."""
    monkeypatch.setenv("TFOCUS_ZVARIANT", str(zvariant))
    g, st = transverse_state(40 + zvariant, (512, 8, 16), 0.3)
    st = st.astype(np.float32).astype(np.float64)
    out, _ = run_gpu(g, "f32", st, 2, 0.41)
    Eo, Bo = psatd.step_fft(st[:3], st[3:], spacing(g), 0.41, nsteps=2)
    assert rel(out.astype(np.float64), np.concatenate([Eo, Bo])) <= 2 * F32_TOL


@pytest.mark.parametrize("zvariant", [7, 9, 10, 11])
def test_long_run_of_512_point_z_kernels_matches_oracle_jump(zvariant, monkeypatch):
    """300 float32 steps with phases c |k| dt up to 7.8 rad per step (where
    variant 10 builds the phase in float32) against the oracle's single exact
    jump (Sec. II.A).  A phase that errs the same way on every step would grow
    linearly with the step count; float32 rounding of the transforms grows as
    a random walk, and the gate is sqrt(steps) times the one-step tolerance."""
    monkeypatch.setenv("TFOCUS_ZVARIANT", str(zvariant))
    g, st = transverse_state(71, (512, 8, 16), 0.3)
    st = st.astype(np.float32).astype(np.float64)
    steps, dt = 300, 0.43
    out, t = run_gpu(g, "f32", st, steps, dt)
    Eo, Bo = psatd.jump(st[:3], st[3:], spacing(g), steps * dt)
    e = rel(out.astype(np.float64), np.concatenate([Eo, Bo]))
    print(f"z variant {zvariant}: {steps} steps vs jump {e:.2e}")
    assert t == pytest.approx(steps * dt)
    assert e <= math.sqrt(steps) * F32_TOL


@pytest.mark.parametrize("zvariant", [7, 8, 9, 10, 11])
def test_wave_z_kernel_projection_and_huge_phases(zvariant, monkeypatch):
    """The one-wave-per-mode z kernel on 512-point columns: the first step
    after tf_set_pulse (which also removes longitudinal B) against the
    oracle's step with the same projection, and a step of unstructured fields
    (longitudinal E present) with phases c |k| dt up to 1e5 rad."""
    monkeypatch.setenv("TFOCUS_ZVARIANT", str(zvariant))
    p = configs.pulse(envelope="spectral", bandwidth=0.4, R0=4.0, L=3.0, f_number=0.5, nfreq=64, cep=0.7)
    g = pulse.layer_grid(p, (32, 16, 512), (0.2, 0.2, 0.2))
    with tf.Solver(g, "f32") as s:
        s.set_pulse(p)
        init = np.empty(s.shape, np.float32)
        s.get_fields(init)
        s.advance(1, 0.37)
        out = np.empty(s.shape, np.float32)
        s.get_fields(out)
    x = init.astype(np.float64)
    Eo, Bo = psatd.step_fft(x[:3], x[3:], spacing(g), 0.37, project_b_first=True)
    assert np.abs(x).max() > 0.1
    assert rel(out.astype(np.float64), np.concatenate([Eo, Bo])) <= F32_TOL
    y = np.random.default_rng(zvariant).standard_normal((6, 512, 16, 32)).astype(np.float32)
    g2 = dict(g, x_min=0.0, y_min=0.0, z_min=0.0)
    out2, _ = run_gpu(g2, "f32", y, 1, 1.0e4)
    Eo, Bo = psatd.step_fft(y[:3].astype(np.float64), y[3:].astype(np.float64), spacing(g2), 1.0e4)
    assert rel(out2.astype(np.float64), np.concatenate([Eo, Bo])) <= F32_TOL


@pytest.mark.parametrize("shape", [(64, 64, 64), (128, 128, 128), (192, 192, 192), (256, 256, 256),
                                   (512, 64, 64), (96, 512, 32)])
def test_y_strip_width_32_keeps_parity(shape, monkeypatch):
    """The fast y kernel on 256-byte strips (32 columns), which the tuner may
    pick instead of 512-byte ones: forward and inverse y passes around every
    z kernel shape the plans use, two steps against the oracle, including
    512-point y columns."""
    monkeypatch.setenv("TFOCUS_YSTRIP", "32")
    g, st = transverse_state(70 + shape[0] + shape[1], shape, 0.3)
    rb, fast, _, ys = tf.tf_kernel_plan(g, "f32")
    assert fast and ys == 32
    st = st.astype(np.float32).astype(np.float64)
    out, _ = run_gpu(g, "f32", st, 2, 0.41)
    Eo, Bo = psatd.step_fft(st[:3], st[3:], spacing(g), 0.41, nsteps=2)
    assert rel(out.astype(np.float64), np.concatenate([Eo, Bo])) <= 2 * F32_TOL


@pytest.mark.parametrize("shape", [(40, 56, 80), (112, 80, 56), (56, 40, 112)])
def test_radix_5_and_7_lengths_f64_match_the_direct_dft_oracle(shape):
    """Axis lengths with factors 5 and 7 (radix-5 and radix-7 stages in the x
    lane groups and in the generic y and z kernels) against the direct-DFT
    step (oracle O1, no FFT library)."""
    g, st = transverse_state(90 + shape[0], shape, 0.21)
    out, _ = run_gpu(g, "f64", st, 1, 0.53)
    Eo, Bo = psatd.step_direct(st[:3], st[3:], spacing(g), 0.53)
    assert rel(out, np.concatenate([Eo, Bo])) <= F64_TOL


@pytest.mark.parametrize("shape, prec", [((896, 8, 16), "f64"), ((8, 16, 896), "f64"), ((16, 896, 8), "f32"),
                                         ((160, 224, 320), "f32"), ((448, 40, 640), "f32")])
def test_radix_5_and_7_long_axes_match_oracle(shape, prec):
    """The paper's 896-node transverse axes (Sec. III.A, Fig. 4) and other
    5- and 7-smooth lengths on every axis, two steps against the oracle."""
    g, st = transverse_state(95 + shape[1], shape, 0.23)
    if prec == "f32":
        st = st.astype(np.float32).astype(np.float64)
    out, _ = run_gpu(g, prec, st, 2, 0.47)
    Eo, Bo = psatd.step_fft(st[:3], st[3:], spacing(g), 0.47, nsteps=2)
    tol = 1e-11 if prec == "f64" else 2 * F32_TOL
    assert rel(out.astype(np.float64), np.concatenate([Eo, Bo])) <= tol


def test_determinism_bitwise():
    g, st = transverse_state(23, (64, 64, 64), 0.25)
    a, _ = run_gpu(g, "f32", st.astype(np.float32), 3, 0.4)
    b, _ = run_gpu(g, "f32", st.astype(np.float32), 3, 0.4)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("n", [64, 128, 192, 256])
@pytest.mark.parametrize("zvariant", [0, 1, 2, 3, 4, 5, 6, 7, 8])
@pytest.mark.parametrize("row_block", ["8", "n"])
def test_every_kernel_plan_keeps_parity(n, zvariant, row_block, monkeypatch):
    """Each z strip shape and y row blocking the tuner can pick."""
    monkeypatch.setenv("TFOCUS_ZVARIANT", str(zvariant))
    monkeypatch.setenv("TFOCUS_ROW_BLOCK", str(n) if row_block == "n" else row_block)
    d = 0.3
    g, st = transverse_state(n + zvariant, (n, n, n), d)
    st = st.astype(np.float32).astype(np.float64)
    out, _ = run_gpu(g, "f32", st, 2, 0.41)
    Eo, Bo = psatd.step_fft(st[:3], st[3:], spacing(g), 0.41, nsteps=2)
    assert rel(out.astype(np.float64), np.concatenate([Eo, Bo])) <= 2 * F32_TOL


@pytest.mark.parametrize("n,row_block", [(128, 16), (192, 64), (256, 32)])
def test_row_blocks_wider_than_the_y_kernel_steps(n, row_block, monkeypatch):
    """Row blocks that do not divide the fast y kernel's row steps, where it
    looks every row up instead of stepping linearly (and the z kernels read
    the wider blocks)."""
    monkeypatch.setenv("TFOCUS_ROW_BLOCK", str(row_block))
    plan = tf.tf_kernel_plan(dict(nx=n, ny=n, nz=n, dx=0.3, dy=0.3, dz=0.3, x_min=0.0, y_min=0.0, z_min=0.0), "f32")
    assert plan[0] == row_block and plan[1]
    g, st = transverse_state(n + row_block, (n, n, n), 0.3)
    st = st.astype(np.float32).astype(np.float64)
    out, _ = run_gpu(g, "f32", st, 2, 0.41)
    Eo, Bo = psatd.step_fft(st[:3], st[3:], spacing(g), 0.41, nsteps=2)
    assert rel(out.astype(np.float64), np.concatenate([Eo, Bo])) <= 2 * F32_TOL


@pytest.mark.parametrize("zvariant", [7, 8])
def test_wave_z_kernel_at_length_256_long_run_and_huge_phases(zvariant, monkeypatch):
    """The one-wave-per-mode z kernel on 256-point columns (radix 4, then the
    64-point lane transform over component pairs): 300 float32 steps against
    the oracle's single exact jump (Sec. II.A), and one step with phases
    c |k| dt up to 1e5 rad on fields with a longitudinal part."""
    monkeypatch.setenv("TFOCUS_ZVARIANT", str(zvariant))
    g, st = transverse_state(130 + zvariant, (256, 16, 32), 0.3)
    st = st.astype(np.float32).astype(np.float64)
    steps, dt = 300, 0.43
    out, _ = run_gpu(g, "f32", st, steps, dt)
    Eo, Bo = psatd.jump(st[:3], st[3:], spacing(g), steps * dt)
    e = rel(out.astype(np.float64), np.concatenate([Eo, Bo]))
    print(f"z variant {zvariant} at 256: {steps} steps vs jump {e:.2e}")
    assert e <= math.sqrt(steps) * F32_TOL
    y = np.random.default_rng(zvariant).standard_normal((6, 256, 16, 32)).astype(np.float32)
    out2, _ = run_gpu(g, "f32", y, 1, 1.0e4)
    Eo, Bo = psatd.step_fft(y[:3].astype(np.float64), y[3:].astype(np.float64), spacing(g), 1.0e4)
    assert rel(out2.astype(np.float64), np.concatenate([Eo, Bo])) <= F32_TOL
