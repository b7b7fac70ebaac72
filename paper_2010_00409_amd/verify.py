"""The method against direct computation (Sec. III.A), the paper's focusing
examples (Sec. III.B.1-2) and the transverse duplication it proposes
(Sec. II.C, closing remarks), on the library.

The paper verifies the mapping on its most demanding case: a flat-top pulse
of f-number 0.3 (opening angle about 1 rad), length L = 2 wavelengths, edge
width 0.1 rad, launched at R0 = 16 wavelengths, advanced to the focus by one
exact step of dt = R0 / c (Sec. II.A: one step of any length is exact).
The direct computation holds the whole pulse in a cube; the method holds it
in a periodic layer of period D along x (Sec. II.C) and cuts the primary
pulse out through Eqs. (14)-(16).  The error is the largest field
difference at the focus relative to the direct computation's peak
(Sec. III.A); the paper reports it against D / L (Fig. 4a) together with
the time and memory the layer saves.

Both runs go through the same C ABI (init on the sphere + mapping, one
spectral step, cut-out); the direct cube is simply a layer whose period
exceeds the pulse's whole x-extent, so every node has one preimage.  Both
windows are read through the same cut-out, so the comparison covers the
region the method returns.
"""
import math
import time

from . import tfocus as tf

# Sec. III.A: f = 0.3, L = 2 lambda, eps = 0.1, R0 = 16 lambda, the paper's
# cos^2 envelope (Eq. (7)) and flat-top aperture (Eq. (5)).
VERIFY_PULSE = dict(envelope="cos2", transverse="flattop", polarization="linear", wavelength=1.0,
                    R0=16.0, L=2.0, ncycles=2.0, f_number=0.3, theta=0.0, eps=0.1, P0=1.0,
                    pol_angle=0.0, ellipticity=0.0, cep=0.0, gdd=0.0, tod=0.0, bandwidth=1.0 / 3.0,
                    nfreq=256)


def cube(n, d):
    return dict(nx=n, ny=n, nz=n, dx=d, dy=d, dz=d, x_min=-(n // 2) * d, y_min=-(n // 2) * d,
                z_min=-(n // 2) * d)


def device_bytes(grid, precision):
    """State plus half spectrum of a solver: 12 elements per node."""
    es = 8 if precision == "f64" else 4
    return 12 * grid["nx"] * grid["ny"] * grid["nz"] * es


def focal_run(grid, pulse, window, precision="f32", reps=3):
    """Focal window after init + one jump of dt = R0 (device tensor) and the
    median seconds of that whole route (init, step, cut-out)."""
    import torch
    dtype = torch.float64 if precision == "f64" else torch.float32
    out = torch.empty((6, window["wz"], window["wy"], window["wx"]), dtype=dtype, device="cuda")
    ts = []
    with tf.Solver(grid, precision, torch.cuda.current_stream()) as s:
        for k in range(reps + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.set_pulse(pulse)
            s.advance(1, float(pulse["R0"]))
            s.read_focal(window, out)
            torch.cuda.synchronize()
            if k:
                ts.append(time.perf_counter() - t0)
    ts.sort()
    return out, ts[len(ts) // 2]


def mapped_vs_direct(layer_nx, points_per_lambda=12, side=512, window=64, precision="f32", pulse=None,
                     reps=3):
    """Errors, times and memory of periodic layers of layer_nx nodes along x
    against the direct cube of side^3 nodes, all at dx = lambda / ppl.
    Returns a dict with one entry per layer."""
    import torch
    p = dict(VERIFY_PULSE if pulse is None else pulse)
    d = float(p["wavelength"]) / points_per_lambda
    win = dict(wx=window, wy=window, wz=window, cx=0.0, cy=0.0, cz=0.0)
    geo = tf.tf_pulse_geometry(p)
    direct = cube(side, d)
    if not side * d / 2 > geo["R_max"]:
        raise ValueError("the direct cube must hold the whole pulse")
    ref, t_direct = focal_run(direct, p, win, precision, reps)
    peak = float(ref.abs().max())
    rows = []
    for nx in layer_nx:
        g = tf.tf_layer_grid(p, (nx, side, side), (d, d, d))
        got, t = focal_run(g, p, win, precision, reps)
        diff = (got.double() - ref.double())
        D = nx * d
        rows.append(dict(nx=nx, D=D, D_over_L=D / p["L"], overlap=D < geo["D_min"],
                         max_err_over_peak=float(diff.abs().max()) / peak,
                         rel_l2=float(diff.norm() / ref.double().norm()),
                         seconds=t, time_ratio=t_direct / t,
                         bytes=device_bytes(g, precision),
                         memory_ratio=device_bytes(direct, precision) / device_bytes(g, precision)))
        del got, diff
    return dict(pulse=p, precision=precision, points_per_lambda=points_per_lambda, side=side, window=window,
                D_min=geo["D_min"], D_min_over_L=geo["D_min"] / p["L"], direct_seconds=t_direct,
                direct_bytes=device_bytes(direct, precision), peak=peak, layers=rows)


# ---------------------------------------------------------------- intensity scans
def intensity_scan(grid, pulse, window, t0, t1, dt, precision="f32", follow=False):
    """Peak of |E|^2 over a window and over the times t0, t0 + dt, ... <= t1
    (one exact jump to t0, then steps of dt), read through the cut-out.  With
    follow the window centre moves with the pulse centre along the axis,
    x = t - R0.  Returns (peak |E|^2, time of the peak, node (x, y, z) of the
    peak).  Every node's field oscillates at the carrier, so with a few
    dozen snapshots per period the largest |E|^2 is the squared amplitude."""
    import numpy as np
    dtype = np.float64 if precision == "f64" else np.float32
    w = np.empty((6, window["wz"], window["wy"], window["wx"]), dtype=dtype)
    best = (-1.0, 0.0, (0.0, 0.0, 0.0))
    n = int(math.floor((t1 - t0) / dt + 1e-9)) + 1
    with tf.Solver(grid, precision) as s:
        s.set_pulse(pulse)
        s.advance(1, t0)
        for k in range(n):
            t = t0 + k * dt
            win = dict(window, cx=window["cx"] + (t - pulse["R0"] if follow else 0.0))
            s.read_focal(win, w)
            e2 = (w[:3].astype(np.float64) ** 2).sum(axis=0)
            i = int(np.argmax(e2))
            if e2.flat[i] > best[0]:
                iz, iy, ix = np.unravel_index(i, e2.shape)
                ic = math.floor((win["cx"] - grid["x_min"]) / grid["dx"] + 0.5)
                jc = math.floor((win["cy"] - grid["y_min"]) / grid["dy"] + 0.5)
                kc = math.floor((win["cz"] - grid["z_min"]) / grid["dz"] + 0.5)
                pos = (grid["x_min"] + (ic + ix - win["wx"] // 2) * grid["dx"],
                       grid["y_min"] + (jc + iy - win["wy"] // 2) * grid["dy"],
                       grid["z_min"] + (kc + iz - win["wz"] // 2) * grid["dz"])
                best = (float(e2.flat[i]), t, pos)
            if k + 1 < n:
                s.advance(1, dt)
    return best


def intensity(e2_peak):
    """Cycle-averaged intensity of a field of squared amplitude |E|^2:
    |E|^2 / (8 pi) (c = 1, the paper's CGS form; the library's amplitude
    makes the cycle-averaged power through the sphere P0)."""
    return e2_peak / (8.0 * math.pi)


# ---------------------------------------------------------------- Sec. III.B.1
# Gaussian temporal and angular profiles: u_l = sin(k zeta) exp(-zeta^2 ln 4 /
# (n lambda)^2) with n = 4 wavelengths (intensity FWHM), u_ts =
# exp(-theta^2 / theta0^2) with tan theta0 = 1 / (2 f), R0 = 20 lambda,
# P0 = 1, on 512 nodes over 40 lambda per axis.  The envelope is cut at
# |zeta| <= L / 2 = 10 lambda, where it has fallen to 1.7e-4.
GAUSS_PULSE = dict(VERIFY_PULSE, envelope="gauss", transverse="gauss", R0=20.0, L=20.0, ncycles=4.0,
                   f_number=1.0)


def paraxial_peak_intensity(f_number, P0=1.0, wavelength=1.0):
    """Peak intensity of a paraxial Gaussian beam of power P0 focused at
    f-number f: I0 = 2 P0 / (pi w0^2) with waist w0 = 2 f lambda / pi
    (Sec. III.B.1)."""
    w0 = 2.0 * f_number * wavelength / math.pi
    return 2.0 * P0 / (math.pi * w0 * w0)


def gaussian_beam_vs_paraxial(f_numbers, n=512, side=40.0, window=48, span=1.0, dt=1.0 / 32, precision="f32",
                              pulse=None):
    """Peak intensity at the focus of the Gaussian beam of Sec. III.B.1 for
    each f-number (times R0 - span ... R0 + span), the paraxial prediction
    and their ratio."""
    rows = []
    base = dict(GAUSS_PULSE if pulse is None else pulse)
    for f in f_numbers:
        p = dict(base, f_number=float(f))
        d = side / n
        g = tf.tf_layer_grid(p, (n, n, n), (d, d, d))
        win = dict(wx=window, wy=window, wz=window, cx=0.0, cy=0.0, cz=0.0)
        e2, t, pos = intensity_scan(g, p, win, p["R0"] - span, p["R0"] + span, dt, precision)
        I, I0 = intensity(e2), paraxial_peak_intensity(f, p["P0"], p["wavelength"])
        rows.append(dict(f_number=float(f), peak_intensity=I, paraxial=I0, ratio=I / I0, t_peak=t,
                         peak_position=list(pos)))
    return rows


# ---------------------------------------------------------------- Sec. III.B.2
def flattop_peak_vs_f(f_numbers, nx=128, nt=1024, window=(64, 48, 48), t_span=(-10.0, 4.0), dt=1.0 / 32,
                      precision="f32", pulse=None):
    """Peak cycle-averaged intensity of the flat-top pulse of Sec. III.A
    (L = 2, eps = 0.1, R0 = 16, P0 = 1) and where and when it is reached, for
    each f-number, in a layer of D = 2 L (Sec. III.B.2: the scheme's error
    stays under 1% of the peak there) of nx nodes along x and nt x nt
    transversely at equal spacing.  The window follows the pulse centre along
    the axis from t = R0 + t_span[0] to R0 + t_span[1]."""
    rows = []
    base = dict(VERIFY_PULSE if pulse is None else pulse)
    for f in f_numbers:
        p = dict(base, f_number=float(f))
        d = 2.0 * p["L"] / nx
        g = tf.tf_layer_grid(p, (nx, nt, nt), (d, d, d))
        win = dict(wx=window[0], wy=window[1], wz=window[2], cx=0.0, cy=0.0, cz=0.0)
        e2, t, pos = intensity_scan(g, p, win, p["R0"] + t_span[0], p["R0"] + t_span[1], dt, precision,
                                    follow=True)
        rows.append(dict(f_number=float(f), theta=tf.tf_pulse_geometry(p)["theta"], peak_intensity=intensity(e2),
                         t_peak=t, x_peak=pos[0], peak_position=list(pos)))
    return rows


# ---------------------------------------------------------------- Sec. II.C, closing remarks
def transverse_duplication(boxes, nx=128, points_per_lambda=12, full=512, window=64, precision="f32",
                           pulse=None, reps=3):
    """The layer shrunk transversely as well: the pulse is replicated along y
    and z with periods ny dy, nz dz (solver periodicity and linearity), so a
    box of n_t x n_t transverse nodes replaces the full_ x full_ one.  Error
    of each box's focal window (one exact step to the focus, through the
    cut-out) against the full transverse layer of the same period, with the
    time and memory the box saves."""
    p = dict(VERIFY_PULSE if pulse is None else pulse)
    d = float(p["wavelength"]) / points_per_lambda
    win = dict(wx=window, wy=window, wz=window, cx=0.0, cy=0.0, cz=0.0)
    ref_grid = tf.tf_layer_grid(p, (nx, full, full), (d, d, d))
    ref, t_ref = focal_run(ref_grid, p, win, precision, reps)
    peak = float(ref.abs().max())
    rows = []
    for nt in boxes:
        g = dict(tf.tf_layer_grid(p, (nx, nt, nt), (d, d, d)), replicate_yz=1)
        got, t = focal_run(g, p, win, precision, reps)
        diff = got.double() - ref.double()
        rows.append(dict(n_t=nt, period=nt * d, period_over_L=nt * d / p["L"],
                         max_err_over_peak=float(diff.abs().max()) / peak,
                         rel_l2=float(diff.norm() / ref.double().norm()), seconds=t, time_ratio=t_ref / t,
                         memory_ratio=device_bytes(ref_grid, precision) / device_bytes(g, precision)))
        del got, diff
    return dict(pulse=p, precision=precision, nx=nx, full=full, reference_seconds=t_ref, peak=peak, boxes=rows)


# ---------------------------------------------------------------- Sec. III.B.3
def phase_bumps(theta, eps_phi, rng, width_frac=0.3):
    """The wavefront perturbation of Sec. III.B.3: (2 theta / sigma)^2 = 44
    Gaussian bumps of width sigma = 0.3 theta, centred uniformly over the
    aperture disc of angular radius theta, amplitudes uniform in
    [-eps_phi, eps_phi].  Returns [(ay, az, amplitude, width)]."""
    sigma = width_frac * theta
    n = int(round((2.0 * theta / sigma) ** 2))
    r = theta * (rng.uniform(size=n) ** 0.5)
    a = 2.0 * math.pi * rng.uniform(size=n)
    amp = rng.uniform(-eps_phi, eps_phi, size=n)
    return [(float(r[i] * math.cos(a[i])), float(r[i] * math.sin(a[i])), float(amp[i]), sigma) for i in range(n)]


def phase_std(bumps, theta, n=201):
    """Standard deviation of the perturbation phase over the aperture disc
    (angular positions |a| <= theta, uniform weight)."""
    import numpy as np
    g = np.linspace(-theta, theta, n)
    ay, az = np.meshgrid(g, g, indexing="ij")
    inside = ay * ay + az * az <= theta * theta
    ph = np.zeros_like(ay)
    for by, bz, amp, w in bumps:
        ph += amp * np.exp(-((ay - by) ** 2 + (az - bz) ** 2) / (w * w))
    return float(ph[inside].std())


def perturbed_focus(eps_values, runs=20, f_number=1.0, nx=96, nt=512, window=(64, 64, 64), t_span=(-2.5, 1.0),
                    dt=1.0 / 32, precision="f32", seed=20100409):
    """Peak cycle-averaged intensity at the focus of the flat-top pulse of
    Sec. III.A (L = 2, eps = 0.1, R0 = 16) at f-number 1 under random
    wavefront perturbations (Sec. III.B.3): for each level eps_phi, runs
    independent draws of phase_bumps, each scanned from R0 + t_span[0] to
    R0 + t_span[1] with the window following the pulse centre, in a D = 2 L
    layer of nx x nt x nt nodes.  Each run is reported as the phase spread
    sigma(phi) over the aperture and the peak intensity relative to the
    unperturbed pulse's."""
    import numpy as np
    rng = np.random.default_rng(seed)
    base = dict(VERIFY_PULSE, f_number=float(f_number))
    theta = tf.tf_pulse_geometry(base)["theta"]
    d = 2.0 * base["L"] / nx
    grid = tf.tf_layer_grid(base, (nx, nt, nt), (d, d, d))
    win = dict(wx=window[0], wy=window[1], wz=window[2], cx=0.0, cy=0.0, cz=0.0)

    def peak(p):
        return intensity_scan(grid, p, win, p["R0"] + t_span[0], p["R0"] + t_span[1], dt, precision, follow=True)

    e2_ref, t_ref, pos_ref = peak(base)
    levels, samples = [], []
    for eps in eps_values:
        ratios, stds = [], []
        for _ in range(runs):
            bumps = phase_bumps(theta, eps, rng)
            e2, _, _ = peak(dict(base, bumps=bumps))
            stds.append(phase_std(bumps, theta))
            ratios.append(e2 / e2_ref)
            samples.append(dict(eps_phi=float(eps), phase_std=stds[-1], intensity_ratio=ratios[-1]))
        levels.append(dict(eps_phi=float(eps), phase_std=float(np.mean(stds)), ratio_mean=float(np.mean(ratios)),
                           ratio_std=float(np.std(ratios)), ratio_min=float(np.min(ratios)), runs=runs))
    return dict(theta=theta, nbumps=len(phase_bumps(theta, 0.0, rng)), peak_intensity=intensity(e2_ref),
                t_peak=t_ref, x_peak=pos_ref[0], levels=levels, samples=samples)
