"""Pins of the oracle's pulse initialisation, mapping and cut-out
(Sec. II.B, II.C, III.A, III.B.1) against closed forms, geometry, brute
force and the paper's printed numbers."""
import math

import numpy as np
import pytest
import scipy.integrate

from oracle import mapping, psatd, pulse
from synthetic import configs


# --- angles and profiles ----------------------------------------------------

def test_theta_from_f_number_matches_configs_in_degrees():
    assert pulse.theta_of(configs.pulse(f_number=0.5)) == pytest.approx(math.pi / 4, abs=1e-15)
    assert math.degrees(pulse.theta_of(configs.pulse(f_number=1.0))) == pytest.approx(26.565, abs=1e-3)
    assert pulse.theta_of(configs.pulse(f_number=0.3)) == pytest.approx(1.0, abs=0.04)  # "theta ~ 1"
    assert pulse.theta_of(configs.pulse(theta=0.9)) == 0.9


def test_flat_top_profile_special_values():
    p = configs.pulse(theta=1.0, eps=0.1)
    g = pulse.geometry(p)
    a = np.array([0.0, 0.5, 0.95 - 1e-12, 0.95, 1.0, 1.05, 1.2])
    v = pulse.u_ts(a, p, g)
    assert list(v[:3]) == [1.0, 1.0, 1.0]
    assert v[3] == pytest.approx(1.0, abs=1e-15)       # edge start, continuous
    assert v[4] == pytest.approx(0.5, abs=1e-15)       # cos^2(pi/4) at theta
    assert v[5] == pytest.approx(0.0, abs=1e-15) and v[6] == 0.0
    fine = np.linspace(0.9, 1.1, 2001)
    assert np.all(np.diff(pulse.u_ts(fine, p, g)) <= 1e-15)   # monotone


def test_gaussian_envelope_has_n_cycle_intensity_fwhm():
    n = 2.0
    p = configs.pulse(envelope="gauss", ncycles=n, L=40.0)
    z = 0.5 * n
    phase = 2 * math.pi * z - math.pi / 2          # carrier peak at zeta = z
    assert pulse.u_l(z, p, phase) ** 2 == pytest.approx(0.5, rel=1e-13)
    assert pulse.u_l(0.0, p, -math.pi / 2) == pytest.approx(1.0, rel=1e-15)


def test_cos2_envelope_vanishes_outside_and_at_edges():
    p = configs.pulse(envelope="cos2", L=2.0)
    z = np.array([-1.5, -1.0, 0.0, 1.0, 1.5])
    assert np.abs(pulse.u_l(z, p, 0.0)).max() < 1e-15
    assert pulse.u_l(0.25, p, 0.0) == pytest.approx(math.cos(math.pi / 8) ** 2, rel=1e-14)


@pytest.mark.parametrize("t0", [0.2, 0.3, 0.5])
def test_F_theta0_residual_is_the_next_taylor_term(t0):
    """Extending the integral to infinity, int_0^inf a^(2n+1) exp(-b a^2) da =
    n!/(2 b^(n+1)) with b = 2/theta0^2 gives the paper's three terms plus
    -theta0^8/26880 + O(theta0^10)."""
    series = t0 ** 2 / 4 - t0 ** 4 / 48 + t0 ** 6 / 960
    resid = (pulse.F_gauss(t0) - series) / t0 ** 8
    assert resid == pytest.approx(-1.0 / 26880.0, rel=0.01)


@pytest.mark.parametrize("t0", [0.5, 1.0, 2.0])
def test_F_theta0_series_is_good_below_two(t0):
    series = t0 ** 2 / 4 - t0 ** 4 / 48 + t0 ** 6 / 960
    assert pulse.F_gauss(t0) == pytest.approx(series, rel=0.012)


# --- fields on the sphere -----------------------------------------------------

def sample_points(rng, n, g):
    R = rng.uniform(g["R_min"], g["R_max"], n)
    al = rng.uniform(0, g["alpha_max"], n)
    ph = rng.uniform(0, 2 * math.pi, n)
    return -R * np.cos(al), R * np.sin(al) * np.cos(ph), R * np.sin(al) * np.sin(ph)


@pytest.mark.parametrize("pol", ["linear", "radial"])
def test_fields_are_transverse_equal_and_point_to_the_focus(pol):
    p = configs.pulse(polarization=pol, pol_angle=0.3)
    g = pulse.geometry(p)
    x, y, z = sample_points(np.random.default_rng(1), 4000, g)
    E, B = pulse.fields_at(x, y, z, p, g)
    R = np.stack([x, y, z])
    big = np.linalg.norm(E, axis=0) > 1e-8
    assert big.sum() > 1000
    assert np.abs((E * R).sum(0)).max() < 1e-12 * np.abs(E).max() * g["R_max"]
    assert np.abs((B * R).sum(0)).max() < 1e-12 * np.abs(B).max() * g["R_max"]
    assert np.abs((E * B).sum(0)).max() < 1e-12 * np.abs(E).max() ** 2
    assert np.allclose(np.linalg.norm(E, axis=0), np.linalg.norm(B, axis=0), rtol=1e-12, atol=1e-14)
    S = np.cross(E.T, B.T).T
    assert np.all((S * R).sum(0)[big] < 0)          # Poynting vector -> focus


def test_linear_polarisation_on_axis_is_y_with_z_magnetic_field():
    p = configs.pulse(cep=0.0)
    g = pulse.geometry(p)
    E, B = pulse.fields_at(-16.25, 0.0, 0.0, p, g)
    assert abs(E[0]) + abs(E[2]) < 1e-15 and abs(B[0]) + abs(B[1]) < 1e-15
    assert E[1] == pytest.approx(B[2], rel=1e-15) and abs(E[1]) > 0


def test_radial_polarisation_vanishes_on_axis_and_is_azimuthal_in_B():
    p = configs.pulse(polarization="radial")
    g = pulse.geometry(p)
    E, B = pulse.fields_at(-16.0, 0.0, 0.0, p, g)
    assert np.abs(E).max() == 0.0 and np.abs(B).max() == 0.0
    E, B = pulse.fields_at(-15.0, 3.0, 0.0, p, g)
    assert abs(B[0]) < 1e-15 and abs(B[1]) < 1e-15 and abs(B[2]) > 0


def test_circular_polarisation_is_in_quadrature():
    p = configs.pulse(envelope="gauss", ncycles=4.0, L=12.0, ellipticity=1.0)
    g = pulse.geometry(p)
    zs = np.linspace(-0.5, 0.5, 201)
    E, _ = pulse.fields_at(-(16.0 + zs), 0 * zs, 0 * zs, p, g)
    amp2 = E[1] ** 2 + E[2] ** 2          # sin^2 + cos^2 of the carrier
    env = np.exp(-2 * zs ** 2 * math.log(4) / 16.0) * g["A"] ** 2 / 2 / (16.0 + zs) ** 2
    assert np.allclose(amp2, env, rtol=1e-12)


def test_pulse_lies_only_in_the_x_negative_sector():
    p = configs.pulse(theta=1.0)
    g = pulse.geometry(p)
    rng = np.random.default_rng(2)
    x, y, z = (rng.uniform(-17, 17, 20000) for _ in range(3))
    E, _ = pulse.fields_at(x, y, z, p, g)
    R = np.sqrt(x * x + y * y + z * z)
    alpha = np.arccos(np.clip(-x / R, -1, 1))
    nonzero = np.linalg.norm(E, axis=0) > 0
    assert np.all(alpha[nonzero] <= 1.05 + 1e-12)
    assert np.all(x[nonzero] < 0)


def test_P11_initial_energy_matches_closed_form():
    """Sum (E^2 + B^2) dV = 2 A^2 Omega_ts int u_l^2 dzeta (the 1/R^2 of u^2
    cancels R^2 dR), Omega_ts = 2 pi int u_ts^2 sin(a) da; with eps -> 0 the
    cycle-averaged power through the cap is A^2 (1 - cos theta) / 4 = P0."""
    p = configs.pulse(envelope="cos2", R0=6.0, L=2.0, theta=0.8, eps=0.1, P0=2.0)
    g = pulse.geometry(p)
    d = 1.0 / 16.0
    n = (96, 224, 224)
    grid = dict(nx=n[0], ny=n[1], nz=n[2], dx=d, dy=d, dz=d,
                x_min=-7.5, y_min=-7.0, z_min=-7.0)
    E, B = pulse.init_fields(p, grid)
    W = float((E ** 2).sum() + (B ** 2).sum()) * d ** 3
    th, eps = 0.8, 0.1

    def uts(a):
        if a < th - eps / 2:
            return 1.0
        if a <= th + eps / 2:
            return math.cos(math.pi * (a - th + eps / 2) / (2 * eps)) ** 2
        return 0.0
    Om = 2 * math.pi * scipy.integrate.quad(lambda a: uts(a) ** 2 * math.sin(a), 0, 1.0,
                                            points=[th - eps / 2, th + eps / 2], epsabs=1e-14)[0]
    Iul = scipy.integrate.quad(lambda s: (math.sin(2 * math.pi * s) * math.cos(math.pi * s / 2) ** 2) ** 2,
                               -1, 1, epsabs=1e-14)[0]
    A2 = 4 * 2.0 / (1 - math.cos(th))
    assert g["A"] ** 2 == pytest.approx(A2, rel=1e-14)
    assert W == pytest.approx(2 * A2 * Om * Iul, rel=2e-3)


# --- D_min and the periodic layer ---------------------------------------------

def overlap(D, g, th, pts):
    """Does the sector region shifted by D along x meet the original one?"""
    x, rho = pts
    xs = x - D
    R = np.sqrt(xs * xs + rho * rho)
    al = np.arctan2(rho, -xs)
    return bool(np.any((R >= g["R_min"]) & (R <= g["R_max"]) & (al <= th)))


@pytest.mark.parametrize("th", [0.4, 0.785, 1.0, 1.3])
def test_P12_D_min_equals_brute_force_no_overlap_period(th):
    p = configs.pulse(R0=16.0, L=2.0, theta=th)
    g = pulse.geometry(p)
    R = np.linspace(g["R_min"], g["R_max"], 201)
    A = np.linspace(0, th, 801)
    RR, AA = np.meshgrid(R, A)
    pts = (-(RR * np.cos(AA)).ravel(), (RR * np.sin(AA)).ravel())
    lo, hi = 0.0, 40.0
    for _ in range(40):
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if overlap(mid, g, th, pts) else (lo, mid)
    assert hi == pytest.approx(g["D_min"], abs=0.02)


def test_P12_D_min_over_L_near_papers_printed_value():
    """Loose pin: the paper prints D_min/L ~ 1.9 for f = 0.3, R0 = 16, L = 2;
    Eq. (12) gives 1.70 at theta and 1.92 at theta + eps, so the printed value
    lies within the range spanned by the aperture's edge width."""
    th = pulse.theta_of(configs.pulse(f_number=0.3))
    vals = [pulse.D_min(th + e, 15.0, 17.0) / 2.0 for e in (0.0, 0.05, 0.1)]
    assert vals[0] == pytest.approx(1.70, abs=0.01)
    assert min(vals) <= 1.9 <= max(vals) + 0.05


def test_layer_grid_places_origin_on_a_node_and_spans_D():
    p = configs.pulse(R0=16.0, L=2.0)
    grid = pulse.layer_grid(p, (56, 64, 64), (1 / 8, 1 / 8, 1 / 8))
    assert grid["x_min"] / grid["dx"] == round(grid["x_min"] / grid["dx"])
    assert grid["x_min"] == pytest.approx(-15.0 - 7.0, abs=grid["dx"] / 2)
    assert grid["y_min"] == -4.0


def test_P13_mapping_is_identity_when_the_pulse_fits():
    p = configs.pulse(envelope="cos2", R0=3.0, L=1.0, theta=0.9)
    g = pulse.geometry(p)
    grid = configs.cube_grid(72, 0.125)
    E, B = pulse.init_fields(p, grid)
    x = grid["x_min"] + np.arange(72) * 0.125
    X, Y, Z = x[None, None, :], x[None, :, None], x[:, None, None]
    Ed, Bd = pulse.fields_at(X, Y, Z, p, g)
    assert np.array_equal(E, Ed) and np.array_equal(B, Bd)


def test_mapping_is_periodic_and_translation_equivariant():
    p = configs.pulse(envelope="cos2", R0=6.0, L=2.0, theta=1.0)
    d = 0.25
    grid = pulse.layer_grid(p, (12, 48, 48), (d, d, d))   # D = 3 < D_min: overlap
    E, _ = pulse.init_fields(p, grid)
    D = 12 * d
    E2, _ = pulse.init_fields(p, dict(grid, x_min=grid["x_min"] + D))
    assert np.allclose(E, E2, atol=1e-13)
    E3, _ = pulse.init_fields(p, dict(grid, x_min=grid["x_min"] + d))
    assert np.allclose(np.roll(E, -1, axis=3), E3, atol=1e-13)


def test_overlapping_replicas_superpose():
    p = configs.pulse(envelope="cos2", R0=6.0, L=2.0, theta=1.0)
    g = pulse.geometry(p)
    d = 0.25
    grid = pulse.layer_grid(p, (12, 8, 8), (d, d, d))
    E, _ = pulse.init_fields(p, grid)
    x = grid["x_min"] + np.arange(12) * d
    y = grid["y_min"] + np.arange(8) * d
    ref = np.zeros_like(E)
    for n in range(-10, 11):
        e, _ = pulse.fields_at(x[None, None, :] + n * 12 * d, y[None, :, None], y[:, None, None], p, g)
        ref += e
    assert np.allclose(E, ref, atol=1e-13)


# --- spectral pulse (sampled spectrum) -----------------------------------------------------

def test_spectral_envelope_unchirped_is_a_gaussian_pulse():
    p = configs.pulse(envelope="spectral", bandwidth=1 / 3, L=12.0, cep=0.7)
    z = np.linspace(-4, 4, 801)
    got = pulse.u_l(z, p, p["cep"])
    w0 = 2 * math.pi
    D = w0 / 3
    ref = np.exp(-(D * z) ** 2 / 4) * np.sin(w0 * z - 0.7)
    ref /= np.abs(ref[np.abs(z) <= 6]).max()
    assert np.abs(got - ref).max() < 2e-3
    assert np.abs(got).max() <= 1.0 + 1e-3


def test_spectral_chirp_sign_and_width_match_the_gaussian_integral():
    gdd = 0.5
    p = configs.pulse(envelope="spectral", bandwidth=0.25, L=40.0, gdd=gdd)
    z = np.linspace(-6, 6, 601)
    got = pulse.g_spectral_raw(z, p, 0.0)
    w0 = 2 * math.pi
    D = 0.25 * w0
    a = 1 / D ** 2 - 0.5j * gdd          # int exp(-W^2 a - i W z) dW
    ref = np.real(np.exp(1j * (math.pi / 2 - w0 * z)) * np.sqrt(math.pi / a) * np.exp(-z ** 2 / (4 * a)))
    scale = (got @ ref) / (ref @ ref)
    assert np.abs(got - scale * ref).max() < 1e-6 * np.abs(got).max()
    # up-chirp: local frequency grows with zeta for GDD > 0
    zc = np.linspace(-4, 4, 4001)
    ph = np.unwrap(np.angle(np.exp(1j * (math.pi / 2 - w0 * zc)) * np.exp(-zc ** 2 / (4 * a))))
    inst = -np.gradient(ph, zc)
    assert inst[-100] > inst[100]


# --- cut-out, Eqs. (14)-(16) --------------------------------------------------

def test_indicator_cases():
    Rmin, Rmax = 15.0, 17.0
    ind = lambda x, t: float(mapping.indicator(x, 0.0, 0.0, t, Rmin, Rmax))
    assert ind(-16.0, 0.0) == 1.0 and ind(-14.9, 0.0) == 0.0 and ind(16.0, 0.0) == 0.0
    assert ind(-8.0, 8.0) == 1.0 and ind(-6.9, 8.0) == 0.0
    assert ind(-1.5, 16.0) == 1.0 and ind(-2.5, 16.0) == 0.0     # x < 0: R <= L
    assert ind(0.9, 16.0) == 1.0 and ind(1.1, 16.0) == 0.0       # x >= 0: R <= r
    assert ind(10.0, 26.0) == 1.0 and ind(-10.0, 26.0) == 0.0 and ind(8.9, 26.0) == 0.0


def test_cutout_decides_nodes_on_its_spheres_alike_in_every_grid():
    """At the focus (t = R0) the cut-out keeps R <= L for x < 0 and
    R <= r(t) = L / 2 for x >= 0; with dx = lambda / 12 and L = 2 the axis
    nodes at x = -24 dx and x = +12 dx lie on those spheres.  A cube centred
    on the origin and layers of every period must read the same window
    through the same cut-out (node coordinates are integer offsets from the
    origin node times the spacing), and those nodes are kept (R = L and
    R = r exactly)."""
    p = configs.pulse(envelope="cos2", R0=16.0, L=2.0, f_number=0.3, eps=0.1)
    g = pulse.geometry(p)
    d = 1 / 12
    win = dict(wx=64, wy=64, wz=64, cx=0.0, cy=0.0, cz=0.0)
    cube = configs.cube_grid(64, d)
    ones = np.ones((6, 64, 64, 64))
    ref = mapping.readout(ones, cube, win, p["R0"], g["R_min"], g["R_max"])
    assert ref[0, 32, 32, 32 - 24] == 1.0 and ref[0, 32, 32, 32 - 25] == 0.0
    assert ref[0, 32, 32, 32 + 12] == 1.0 and ref[0, 32, 32, 32 + 13] == 0.0
    for nx in (48, 64, 96, 128, 192):
        grid = pulse.layer_grid(p, (nx, 64, 64), (d, d, d))
        out = mapping.readout(np.ones((6, 64, 64, nx)), grid, win, p["R0"], g["R_min"], g["R_max"])
        assert np.array_equal(out, ref), nx


def test_readout_at_start_recovers_the_unmapped_pulse():
    p = configs.pulse(envelope="cos2", R0=6.0, L=2.0, theta=1.0)
    g = pulse.geometry(p)
    d = 0.125
    grid = pulse.layer_grid(p, (48, 112, 112), (d, d, d))       # D = 6 = 3 L
    E, B = pulse.init_fields(p, grid)
    win = dict(wx=64, wy=104, wz=104, cx=-4.0, cy=0.0, cz=0.0)
    out = mapping.readout(np.concatenate([E, B]), grid, win, 0.0, g["R_min"], g["R_max"])
    I, J, K = mapping.window_nodes(grid, win)
    x = grid["x_min"] + I * d
    y = grid["y_min"] + J * d
    z = grid["z_min"] + K * d
    Ed, Bd = pulse.fields_at(x[None, None, :], y[None, :, None], z[:, None, None], p, g)
    assert np.abs(out - np.concatenate([Ed, Bd])).max() < 1e-12
    assert np.abs(out).max() > 0.1


@pytest.mark.slow
def test_P14_mapped_focus_converges_to_direct_computation():
    """Reduced version of Sec. III.A: theta = 1, L = 2, eps = 0.1, one step
    of dt = R0 to focus; R0 = 8 at 8 points per wavelength.  The error of the
    mapped layer (max |diff| / peak, the paper's metric) must fall with D/L and
    stay at the percent level from D/L ~ 2 on (paper: 0.9% at D_min, <0.1% at
    3.5 L for R0 = 16 at 12 points per wavelength)."""
    p = configs.pulse(envelope="cos2", R0=8.0, L=2.0, theta=1.0, eps=0.1)
    g = pulse.geometry(p)
    d = 1 / 8
    ny = 160
    direct = dict(nx=160, ny=ny, nz=ny, dx=d, dy=d, dz=d, x_min=-12.0,
                  y_min=-(ny // 2) * d, z_min=-(ny // 2) * d)
    win = dict(wx=32, wy=32, wz=32, cx=0.0, cy=0.0, cz=0.0)
    T = p["R0"]

    def focal(grid):
        E, B = pulse.init_fields(p, grid)
        E, B = psatd.step_fft(E, B, (d, d, d), T, 1, project_b_first=True)
        return mapping.readout(np.concatenate([E, B]), grid, win, T, g["R_min"], g["R_max"])
    ref = focal(direct)
    peak = np.abs(ref).max()
    errs = []
    for DL in (1.5, 2.5, 3.5):
        grid = pulse.layer_grid(p, (int(round(DL * 2 / d)), ny, ny), (d, d, d))
        errs.append(np.abs(focal(grid) - ref).max() / peak)
    assert errs[0] > errs[1] > errs[2]
    assert errs[1] < 0.01 and errs[2] < 0.006


def _dup_case():
    p = configs.pulse(envelope="cos2", R0=4.0, L=2.0, theta=0.8, eps=0.1)
    d = 0.25
    big = pulse.layer_grid(p, (16, 48, 48), (d, d, d))        # holds the pulse: |y|, |z| < 6
    small = dict(pulse.layer_grid(p, (16, 16, 16), (d, d, d)), replicate_yz=1)
    return p, d, big, small


def test_transverse_replication_folds_the_full_layer():
    """Duplication along y and z (Sec. II.C closing remarks): the replicated
    init of a 16 x 16 transverse box equals the init of a box holding the
    whole pulse folded onto it (block rows j, j + 16, j + 32 summed), and on
    the box holding the pulse replication adds nothing."""
    p, d, big, small = _dup_case()
    Eb, Bb = pulse.init_fields(p, big)
    Es, Bs = pulse.init_fields(p, small)
    fb = np.concatenate([Eb, Bb])
    fold = sum(fb[:, 16 * l:16 * (l + 1), 16 * m:16 * (m + 1), :] for l in range(3) for m in range(3))
    got = np.concatenate([Es, Bs])
    assert np.abs(fb).max() > 0.1
    assert np.abs(got - fold).max() <= 1e-12 * np.abs(fold).max()
    Er, Br = pulse.init_fields(p, dict(big, replicate_yz=1))
    assert np.array_equal(Er, Eb) and np.array_equal(Br, Bb)


def test_transverse_replication_wraps_the_window():
    """A window wider than the replicated box reads the periodic state: it
    equals the window of the state tiled three times along y and z."""
    p, d, big, small = _dup_case()
    g = pulse.geometry(p)
    st = np.random.default_rng(3).standard_normal((6, 16, 16, 16))
    win = dict(wx=8, wy=24, wz=20, cx=0.0, cy=0.3, cz=-0.2)
    out = mapping.readout(st, small, win, 1.0, g["R_min"], g["R_max"])
    tiled = np.tile(st, (1, 3, 3, 1))
    tg = dict(small, replicate_yz=0, ny=48, nz=48, y_min=small["y_min"] - 16 * d, z_min=small["z_min"] - 16 * d)
    ref = mapping.readout(tiled, tg, win, 1.0, g["R_min"], g["R_max"])
    assert np.array_equal(out, ref)


def test_phase_bump_closed_forms():
    """A single bump of amplitude a and width w centred on the axis gives
    phase a on the axis and a / e at angular distance w (Sec. III.B.3)."""
    p = dict(configs.pulse(), bumps=[(0.0, 0.0, 0.7, 0.2)])
    alpha = np.array([0.0, 0.2, 0.2])
    y = np.array([0.0, 1.0, 0.0])
    z = np.array([0.0, 0.0, -1.0])
    ph = pulse.bump_phase(alpha, y, z, p)
    assert np.allclose(ph, [0.7, 0.7 / np.e, 0.7 / np.e], rtol=1e-14)


@pytest.mark.parametrize("envelope", ["cos2", "spectral"])
def test_uniform_phase_bump_is_a_carrier_phase_shift(envelope):
    """A bump far wider than the aperture adds one constant phase to every
    direction: the perturbed pulse equals the pulse with that phase added to
    its carrier-envelope phase (up to the spectral envelope's normalisation)."""
    p = configs.pulse(envelope=envelope, R0=4.0, L=2.0, theta=0.8, eps=0.1, nfreq=64, cep=0.3)
    grid = pulse.layer_grid(p, (16, 32, 32), (0.25, 0.25, 0.25))
    E1, B1 = pulse.init_fields(dict(p, bumps=[(0.1, -0.2, 0.9, 1e6)]), grid)
    E2, B2 = pulse.init_fields(dict(p, cep=1.2), grid)
    if envelope == "spectral":
        # the sampled-spectrum envelope is normalised by its peak at the
        # pulse's own CEP; a bump leaves that normalisation alone
        s = pulse.spectral_norm(dict(p, cep=1.2)) / pulse.spectral_norm(p)
        E2, B2 = E2 * s, B2 * s
    ref = np.abs(E2).max()
    assert ref > 0.1
    assert np.abs(E1 - E2).max() <= 1e-12 * ref and np.abs(B1 - B2).max() <= 1e-12 * ref


def test_perturbation_draws_follow_the_paper():
    """(2 theta / sigma)^2 = 44 bumps of width 0.3 theta inside the aperture
    disc, amplitudes within +-eps_phi; the phase spread grows with eps_phi."""
    from paper_2010_00409_amd import verify
    rng = np.random.default_rng(0)
    th = 0.4636
    b = verify.phase_bumps(th, 0.5, rng)
    assert len(b) == 44
    assert all(by * by + bz * bz <= th * th + 1e-15 and abs(a) <= 0.5 and w == pytest.approx(0.3 * th)
               for by, bz, a, w in b)
    s1 = verify.phase_std(verify.phase_bumps(th, 0.2, np.random.default_rng(1)), th)
    s2 = verify.phase_std(verify.phase_bumps(th, 0.8, np.random.default_rng(1)), th)
    assert 0 < s1 < s2 and s2 == pytest.approx(4 * s1, rel=1e-12)
