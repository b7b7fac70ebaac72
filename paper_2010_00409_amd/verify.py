"""The method against direct computation (Sec. III.A), on the library.

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
