"""GPU parity of the step with a current held over the step (Sec. II.A,
Eqs. (1)-(2)) through the C ABI against the float64 oracle's
step_fft_current on the same seeded inputs.  Tolerances (relative L2 over
all six components): float64 <= 1e-12, float32 <= 1e-5."""
import numpy as np
import pytest

from oracle import psatd, pulse
from paper_2010_00409_amd import tfocus as tf
from synthetic import configs

pytestmark = pytest.mark.gpu

F64_TOL = 1e-12
F32_TOL = 1e-5


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def spacing(g):
    return (g["dz"], g["dy"], g["dx"])


def inputs(seed, shape, d):
    """Random E (with a longitudinal part), B without magnetic charge and a
    random current on a periodic grid."""
    g = dict(nx=shape[2], ny=shape[1], nz=shape[0], dx=d, dy=0.9 * d, dz=1.1 * d, x_min=0.0, y_min=0.0, z_min=0.0)
    rng = np.random.default_rng(seed)
    E, B, J = (rng.standard_normal((3,) + shape) for _ in range(3))
    _, B = psatd.step_fft(E, B, spacing(g), 0.0, project_b_first=True)
    return g, np.concatenate([E, B]), J


def gpu_current_step(g, prec, state, J, dt, nsteps=1, device_j=False):
    import torch
    dtype = np.float64 if prec == "f64" else np.float32
    with tf.Solver(g, prec) as s:
        s.set_fields(np.ascontiguousarray(state, dtype=dtype), 0.0)
        j = np.ascontiguousarray(J, dtype=dtype)
        if device_j:
            j = torch.from_numpy(j).cuda()
        for _ in range(nsteps):
            s.advance_current(j, dt)
        if device_j:
            torch.cuda.synchronize()
        out = np.empty(s.shape, dtype=dtype)
        s.get_fields(out)
        t = s.t
    return out, t


@pytest.mark.parametrize("shape, dt", [((24, 32, 40), 0.37), ((16, 48, 64), -2.3), ((96, 8, 24), 41.0)])
def test_current_step_f64_matches_oracle(shape, dt):
    g, st, J = inputs(3 + shape[0], shape, 0.25)
    out, t = gpu_current_step(g, "f64", st, J, dt)
    Eo, Bo = psatd.step_fft_current(st[:3], st[3:], J, spacing(g), dt)
    assert rel(out, np.concatenate([Eo, Bo])) <= F64_TOL
    assert t == pytest.approx(dt)


@pytest.mark.parametrize("shape", [(64, 64, 64), (128, 96, 48), (512, 16, 32)])
def test_current_step_f32_matches_oracle(shape):
    """Float32 with the fast x and y kernels around the current z pass, two
    steps with the same current (host and device copies of j)."""
    g, st, J = inputs(11 + shape[0], shape, 0.3)
    st = st.astype(np.float32).astype(np.float64)
    J = J.astype(np.float32).astype(np.float64)
    Eo, Bo = psatd.step_fft_current(st[:3], st[3:], J, spacing(g), 0.41)
    Eo, Bo = psatd.step_fft_current(Eo, Bo, J, spacing(g), 0.41)
    ref = np.concatenate([Eo, Bo])
    host, _ = gpu_current_step(g, "f32", st, J, 0.41, nsteps=2)
    dev, _ = gpu_current_step(g, "f32", st, J, 0.41, nsteps=2, device_j=True)
    assert rel(host.astype(np.float64), ref) <= 2 * F32_TOL
    assert np.array_equal(host, dev)


def test_uniform_current_from_zero_fields_ramps_E():
    g, _, _ = inputs(1, (16, 16, 16), 0.2)
    j0 = np.array([0.3, -1.2, 0.7])
    J = np.broadcast_to(j0[:, None, None, None], (3, 16, 16, 16)).copy()
    out, _ = gpu_current_step(g, "f64", np.zeros((6, 16, 16, 16)), J, 0.45)
    assert np.abs(out[:3] - (-4.0 * np.pi * 0.45) * J).max() <= 1e-13
    assert np.abs(out[3:]).max() <= 1e-13


def test_current_step_after_set_pulse_removes_longitudinal_B_first():
    p = configs.pulse(envelope="spectral", bandwidth=0.4, R0=4.0, L=3.0, f_number=0.5, nfreq=64)
    g = pulse.layer_grid(p, (24, 32, 32), (0.2, 0.2, 0.2))
    rng = np.random.default_rng(4)
    J = rng.standard_normal((3, 32, 32, 24))
    with tf.Solver(g, "f64") as s:
        s.set_pulse(p)
        init = np.empty(s.shape)
        s.get_fields(init)
        s.advance_current(J, 0.3)
        s.advance(1, 0.2)
        out = np.empty(s.shape)
        s.get_fields(out)
    Eo, Bo = psatd.step_fft_current(init[:3], init[3:], J, spacing(g), 0.3, project_b=True)
    Eo, Bo = psatd.step_fft(Eo, Bo, spacing(g), 0.2)
    assert rel(out, np.concatenate([Eo, Bo])) <= F64_TOL


def test_current_step_refuses_what_the_lds_cannot_hold():
    g = dict(nx=8, ny=8, nz=1024, dx=0.1, dy=0.1, dz=0.1, x_min=0.0, y_min=0.0, z_min=0.0)
    with tf.Solver(g, "f64") as s:
        with pytest.raises(tf.TfError) as ei:
            s.advance_current(np.zeros((3, 1024, 8, 8)), 0.1)
        assert ei.value.status == tf.TF_EUNSUPPORTED
        assert s.t == 0.0
