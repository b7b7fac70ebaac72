"""Pins of the oracle's spectral step against what the paper and the
mathematics fix (Sec. II.A, Eqs. (3)-(4)): exact phase advance of plane
waves (zero numerical dispersion), Parseval energy, transversality,
reversibility, the semigroup property of exact steps, special cases,
translation invariance, reality, and the direct DFT against brute force."""
import itertools
import math

import numpy as np
import pytest

from oracle import dft, psatd
from synthetic import configs, planewaves


def closed_form(modes, grid, t):
    """Plane-wave solution of the vacuum Maxwell equations (c = 1):
    E = a e cos(k.x - s|k|t + phi), B = s k_hat x E."""
    x, y, z = planewaves.node_coords(grid)
    shape = (grid["nz"], grid["ny"], grid["nx"])
    E = np.zeros((3,) + shape)
    B = np.zeros((3,) + shape)
    for md in modes:
        k = planewaves.kvec(md, grid)
        w = math.sqrt(k @ k)
        ph = (k[0] * x[None, None, :] + k[1] * y[None, :, None]
              + k[2] * z[:, None, None] - md["sign"] * w * t + md["phase"])
        c = md["amp"] * np.cos(ph)
        kh = k / w
        b = md["sign"] * np.cross(kh, md["e"])
        for a in range(3):
            E[a] += md["e"][a] * c
            B[a] += b[a] * c
    return E, B


def spacing(g):
    return (g["dz"], g["dy"], g["dx"])


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


# --- the direct DFT (O1) -----------------------------------------------------

def test_dftn_matches_brute_force_triple_sum():
    rng = np.random.default_rng(0)
    f = rng.standard_normal((3, 4, 5)) + 1j * rng.standard_normal((3, 4, 5))
    F = dft.dftn(f)
    ref = np.zeros_like(f)
    for m in itertools.product(range(3), range(4), range(5)):
        acc = 0j
        for j in itertools.product(range(3), range(4), range(5)):
            ph = -2 * math.pi * (m[0] * j[0] / 3 + m[1] * j[1] / 4 + m[2] * j[2] / 5)
            acc += f[j] * complex(math.cos(ph), math.sin(ph))
        ref[m] = acc
    assert np.abs(F - ref).max() < 1e-12
    assert np.abs(dft.idftn(F) - f).max() < 1e-13


def test_dftn_of_delta_and_single_exponential():
    f = np.zeros((4, 6, 8))
    f[0, 0, 0] = 1.0
    assert np.allclose(dft.dftn(f), 1.0, atol=1e-15)
    j = np.arange(8)
    e = np.exp(2j * np.pi * 3 * j / 8)[None, None, :] * np.ones((4, 6, 8))
    F = dft.dftn(e)
    expect = np.zeros((4, 6, 8), complex)
    expect[0, 0, 3] = 4 * 6 * 8
    assert np.abs(F - expect).max() < 1e-11


# --- P1/P2: exact plane-wave advance -----------------------------------------

@pytest.mark.parametrize("dt", [0.125, 0.37, -0.21, 13.7])
def test_P1_single_plane_wave_is_advanced_exactly(dt):
    g = configs.cube_grid(32, 0.25)
    modes = planewaves.draw(11, nmodes=1, mmax=15)
    E, B = planewaves.fields(modes, g)
    for s in range(1, 4):
        E, B = psatd.step_fft(E, B, spacing(g), dt)
        Ec, Bc = closed_form(modes, g, s * dt)
        assert np.abs(E - Ec).max() < 1e-12
        assert np.abs(B - Bc).max() < 1e-12


def test_P1_direction_of_propagation_fixes_fft_sign():
    # E = y cos(kx), B = z cos(kx) moves towards +x (forward transform exp(-i k.x)): after a quarter
    # period the field is y sin(kx).
    g = configs.cube_grid(16, 0.25)
    x, _, _ = planewaves.node_coords(g)
    k = 2 * math.pi * 2 / 4.0
    E = np.zeros((3, 16, 16, 16))
    B = np.zeros_like(E)
    E[1] = np.cos(k * x)[None, None, :]
    B[2] = np.cos(k * x)[None, None, :]
    E1, B1 = psatd.step_fft(E, B, spacing(g), 0.25 * 2 * math.pi / k)
    assert np.abs(E1[1] - np.sin(k * x)[None, None, :]).max() < 1e-13
    assert np.abs(B1[2] - np.sin(k * x)[None, None, :]).max() < 1e-13


def test_P2_sixteen_mode_superposition_C1_grid():
    c = configs.c1()
    g = c["grid"]
    modes = planewaves.draw(c["planewave_seed"], nmodes=16, mmax=31)
    E, B = planewaves.fields(modes, g)
    E, B = psatd.step_fft(E, B, spacing(g), c["dt"], nsteps=8)
    Ec, Bc = closed_form(modes, g, 8 * c["dt"])
    assert rel(np.concatenate([E, B]), np.concatenate([Ec, Bc])) < 1e-13


# --- P3..P9 --------------------------------------------------------------------

def transverse_random(seed, n=16, d=0.3):
    g = configs.cube_grid(n, d)
    E, B = planewaves.random_fields(seed, (n, n, n))
    E, B = psatd.step_fft(E, B, spacing(g), 0.0, project_b_first=True)
    return g, E, B


def test_P3_energy_is_conserved():
    g, E, B = transverse_random(3)
    W0 = psatd.energy(E, B)
    for _ in range(10):
        E, B = psatd.step_fft(E, B, spacing(g), 0.77)
        assert abs(psatd.energy(E, B) - W0) < 1e-12 * W0


def test_P4_longitudinal_fields_are_removed():
    g = configs.cube_grid(16, 0.3)
    E, B = planewaves.random_fields(4, (16, 16, 16))
    dE, dB = psatd.max_divergence(E, B, spacing(g))
    assert dE > 0.1 and dB > 0.1
    E1, B1 = psatd.step_fft(E, B, spacing(g), 0.4, project_b_first=False)
    dE1, dB1 = psatd.max_divergence(E1, B1, spacing(g))
    assert dE1 < 1e-13          # Eq. (3) removes k(k.E) every step
    assert dB1 > 0.1            # Eq. (4) alone keeps longitudinal B
    E2, B2 = psatd.step_fft(E, B, spacing(g), 0.4, project_b_first=True)
    assert max(psatd.max_divergence(E2, B2, spacing(g))) < 1e-13


def test_P5_time_reversibility():
    g, E, B = transverse_random(5)
    E1, B1 = psatd.step_fft(E, B, spacing(g), 0.3, nsteps=7)
    E2, B2 = psatd.step_fft(E1, B1, spacing(g), -0.3, nsteps=7)
    assert rel(np.concatenate([E2, B2]), np.concatenate([E, B])) < 1e-13


def test_P6_semigroup_n_steps_equal_one_jump():
    g, E, B = transverse_random(6)
    E1, B1 = psatd.step_fft(E, B, spacing(g), 0.3, nsteps=12)
    E2, B2 = psatd.jump(E, B, spacing(g), 12 * 0.3)
    assert rel(np.concatenate([E1, B1]), np.concatenate([E2, B2])) < 1e-13


def test_P7_dt_zero_is_a_projection_and_full_period_is_identity():
    g = configs.cube_grid(16, 0.3)
    E, B = planewaves.random_fields(7, (16, 16, 16))
    E1, B1 = psatd.step_fft(E, B, spacing(g), 0.0)
    assert np.abs(B1 - B).max() < 1e-13               # C = 1, S = 0
    E2, B2 = psatd.step_fft(E1, B1, spacing(g), 0.0)
    assert np.abs(E2 - E1).max() < 1e-13               # idempotent projection
    modes = planewaves.draw(8, nmodes=1, mmax=7)
    Ep, Bp = planewaves.fields(modes, g)
    k = np.linalg.norm(planewaves.kvec(modes[0], g))
    E3, B3 = psatd.step_fft(Ep, Bp, spacing(g), 2 * math.pi / k)
    assert np.abs(E3 - Ep).max() < 1e-12 and np.abs(B3 - Bp).max() < 1e-12


def test_P8_translation_by_a_node_commutes_with_the_step():
    g, E, B = transverse_random(9)
    sh = lambda a: np.roll(a, (1, -2, 3), axis=(1, 2, 3))
    E1, B1 = psatd.step_fft(sh(E), sh(B), spacing(g), 0.55)
    E2, B2 = psatd.step_fft(E, B, spacing(g), 0.55)
    assert np.abs(E1 - sh(E2)).max() < 1e-13


def test_P9_P10_direct_dft_step_is_real_and_matches_fft_step():
    g = configs.cube_grid(12, 0.4)
    g2 = dict(g, nx=10, x_min=-2.0)
    E, B = planewaves.random_fields(10, (12, 12, 10))
    for kw in ({}, {"project_b": True}):
        E1, B1 = psatd.step_direct(E, B, spacing(g2), 0.9, **kw)   # asserts P9
        E2, B2 = psatd.step_fft(E, B, spacing(g2), 0.9,
                                project_b_first=kw.get("project_b", False))
        assert np.abs(E1 - E2).max() < 1e-13
        assert np.abs(B1 - B2).max() < 1e-13


def test_nyquist_modes_with_signed_reading_would_break_reality():
    # The Nyquist -> 0 reading is what keeps the step real: giving the
    # Nyquist index the value -N/2 produces an O(1) imaginary residue.
    n = 8
    s = psatd.signed_index(n)
    assert s[n // 2] == 0.0 and s[1] == 1.0 and s[-1] == -1.0
    g = configs.cube_grid(n, 0.5)
    E, B = planewaves.random_fields(12, (n, n, n))
    Eh = [dft.dftn(E[a]) for a in range(3)]
    Bh = [dft.dftn(B[a]) for a in range(3)]
    sb = np.where(np.arange(n) < n // 2, np.arange(n), np.arange(n) - n).astype(float)
    kk = 2 * np.pi * sb / (n * 0.5)
    k = (kk[None, None, :], kk[None, :, None], kk[:, None, None])
    En, _ = psatd.update(Eh, Bh, k, 0.7)
    im = max(np.abs(dft.idftn(x).imag).max() for x in En)
    assert im > 1e-3


# ---------------------------------------------------------------- currents
def _cross_matrix(k):
    """K with K v = k x v."""
    return np.array([[0.0, -k[2], k[1]], [k[2], 0.0, -k[0]], [-k[1], k[0], 0.0]])


def _maxwell_mode_exact(k, E, B, J, dt):
    """Exact solution of d/dt E = i c k x B - 4 pi J, d/dt B = -i c k x E
    (CGS, c = 1; Maxwell's curl equations for one Fourier mode with grad ->
    +ik) over dt with J constant: the matrix exponential of the system
    augmented by a constant state."""
    import scipy.linalg
    K = _cross_matrix(k)
    A = np.zeros((7, 7), complex)
    A[0:3, 3:6] = 1j * K
    A[3:6, 0:3] = -1j * K
    A[0:3, 6] = -4.0 * np.pi * J
    y = scipy.linalg.expm(A * dt) @ np.concatenate([E, B, [1.0]])
    return y[0:3], y[3:6]


@pytest.mark.parametrize("dt", [0.013, 0.7, 23.0, -1.9])
def test_current_step_is_the_exact_solution_of_maxwells_equations_per_mode(dt):
    """Eqs. (1)-(2) against the matrix exponential of the curl equations with
    a constant current, for random modes (k = 0 included), complex E (with a
    longitudinal part) and j, and B with k . B = 0 (Eq. (2), like Eq. (4),
    holds for B without magnetic charge: a longitudinal B is constant in
    Maxwell's equations but would be multiplied by C)."""
    rng = np.random.default_rng(11)
    for trial in range(20):
        k = rng.standard_normal(3) * (0.0 if trial == 0 else rng.uniform(0.1, 4.0))
        E, B, J = (rng.standard_normal(3) + 1j * rng.standard_normal(3) for _ in range(3))
        if trial:
            B = B - k * (k @ B) / (k @ k)
        Ee, Be = _maxwell_mode_exact(k, E, B, J, dt)
        kk = tuple(np.array(x) for x in k)
        En, Bn = psatd.update_with_current(list(E), list(B), list(J), kk, dt)
        got = np.concatenate([np.array(En, complex).ravel(), np.array(Bn, complex).ravel()])
        ref = np.concatenate([Ee, Be])
        assert np.abs(got - ref).max() <= 1e-11 * max(1.0, np.abs(ref).max()), (trial, dt)


def test_current_step_semigroup_for_a_constant_current():
    """With the current held constant, two steps of dt equal one of 2 dt
    (Eqs. (1)-(2) are the exact solution over any interval) for B without
    magnetic charge."""
    shape, sp = (8, 10, 12), (0.3, 0.25, 0.2)
    rng = np.random.default_rng(5)
    E, B, J = (rng.standard_normal((3,) + shape) for _ in range(3))
    _, B = psatd.step_fft(E, B, sp, 0.0, project_b_first=True)
    E1, B1 = psatd.step_fft_current(E, B, J, sp, 0.37)
    E2, B2 = psatd.step_fft_current(E1, B1, J, sp, 0.37)
    E3, B3 = psatd.step_fft_current(E, B, J, sp, 0.74)
    ref = np.concatenate([E3, B3])
    assert np.abs(np.concatenate([E2, B2]) - ref).max() <= 1e-12 * np.abs(ref).max()


def test_current_step_without_current_on_transverse_fields_is_the_vacuum_step():
    """j = 0 and div E = 0: Eqs. (1)-(2) reduce to Eqs. (3)-(4)."""
    shape, sp = (8, 10, 12), (0.3, 0.25, 0.2)
    E, B = planewaves.random_fields(3, shape)
    E, B = psatd.step_fft(E, B, sp, 0.0, project_b_first=True)
    Ec, Bc = psatd.step_fft_current(E, B, np.zeros_like(E), sp, 0.9)
    Ev, Bv = psatd.step_fft(E, B, sp, 0.9)
    assert np.abs(np.concatenate([Ec - Ev, Bc - Bv])).max() <= 1e-13


def test_uniform_current_ramps_the_uniform_field():
    """A uniform current from zero fields: E = -4 pi dt j everywhere, B = 0
    (the k = 0 limits S / (kappa c) -> dt, (1 - C) / (kappa c) -> 0)."""
    shape, sp = (6, 8, 10), (0.3, 0.25, 0.2)
    j0 = np.array([0.3, -1.2, 0.7])
    J = np.broadcast_to(j0[:, None, None, None], (3,) + shape).copy()
    Z = np.zeros((3,) + shape)
    E, B = psatd.step_fft_current(Z, Z, J, sp, 0.45)
    assert np.abs(E - (-4.0 * np.pi * 0.45) * J).max() <= 1e-13
    assert np.abs(B).max() <= 1e-13


def test_current_step_keeps_gauss_law_with_charge_continuity():
    """k . (E' - E) = -4 pi dt k . j for every mode: the charge the current
    moves, div E changing by -4 pi dt div j."""
    import scipy.fft
    shape, sp = (8, 10, 12), (0.3, 0.25, 0.2)
    rng = np.random.default_rng(9)
    E, B, J = (rng.standard_normal((3,) + shape) for _ in range(3))
    E1, _ = psatd.step_fft_current(E, B, J, sp, 1.3)
    k = psatd.wavevector(shape, sp, half_x=True)
    dEh = [scipy.fft.rfftn(E1[a] - E[a]) for a in range(3)]
    Jh = [scipy.fft.rfftn(J[a]) for a in range(3)]
    lhs = sum(k[a] * dEh[a] for a in range(3))
    rhs = -4.0 * np.pi * 1.3 * sum(k[a] * Jh[a] for a in range(3))
    assert np.abs(lhs - rhs).max() <= 1e-10 * np.abs(rhs).max()
