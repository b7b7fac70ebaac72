"""Workload recipes: grid sizes, pulse parameters and seeds.

Units: c = 1 and wavelength = 1, so one time unit is lambda/c; for a 1 um
wavelength that is 3.3356 fs, the factor used to express fs-valued chirps.
Everything is synthetic and seeded from ``ROOT_SEED``.

C1  64^3 float64 cube (side 16, centred on the origin), Gaussian envelope of
    2 cycles (intensity FWHM), flat-top aperture 0.9 rad, linear y
    polarisation, shell radius 6; plus 16 random plane waves.
C2  256^3 float32 layer, dx = 1/8, f = 1, one-octave spectral pulse,
    R0 = 25, 400 steps of dt = 1/16, 64^3 focal window.
C3  512^3 float32 layer, dx = 1/12, f = 0.5, two-octave spectral pulse,
    radial polarisation, R0 = 16, 1000 steps of dt = 1/24 (headline).
C4  batched sweep of uneven cubes {128, 192, 256}^3 with random f, CEP, GDD.
C5  surrogate training/test parameter sets (8 parameters per run).
"""
import copy

import numpy as np

ROOT_SEED = 20100409
FS_PER_UNIT = 3.3356409519815204      # lambda / c in fs for lambda = 1 um

BASE_PULSE = dict(envelope="cos2", transverse="flattop", polarization="linear",
                  wavelength=1.0, R0=16.0, L=2.0, ncycles=2.0, f_number=0.3,
                  theta=0.0, eps=0.1, P0=1.0, pol_angle=0.0, ellipticity=0.0,
                  cep=0.0, gdd=0.0, tod=0.0, bandwidth=1.0 / 3.0, nfreq=256)


def pulse(**kw):
    p = copy.deepcopy(BASE_PULSE)
    for k, v in kw.items():
        if k not in p:
            raise KeyError(k)
        p[k] = v
    return p


def cube_grid(n, d):
    """A cube of n^3 nodes centred on the origin (origin is a node)."""
    return dict(nx=n, ny=n, nz=n, dx=d, dy=d, dz=d,
                x_min=-(n // 2) * d, y_min=-(n // 2) * d, z_min=-(n // 2) * d)


def _cep(seed):
    return float(np.random.default_rng(seed).uniform(0.0, 2.0 * np.pi))


def c1():
    """Plain method, float64, 64^3, side 16 (dx = 1/4), 64 steps."""
    return dict(name="C1", n=(64, 64, 64), spacing=(0.25, 0.25, 0.25),
                grid=cube_grid(64, 0.25), precision="f64", dt=0.125, steps=64,
                pulse=pulse(envelope="gauss", ncycles=2.0, L=10.0, R0=6.0,
                            theta=0.9, eps=0.1, transverse="flattop"),
                planewave_seed=1, planewaves=16)


def c2():
    """Plain method, float32, 256^3, dx = 1/8, one-octave pulse, f = 1."""
    return dict(name="C2", n=(256, 256, 256), spacing=(0.125, 0.125, 0.125),
                precision="f32", dt=0.0625, steps=400,
                pulse=pulse(envelope="spectral", bandwidth=1.0 / 3.0, L=8.0,
                            R0=25.0, f_number=1.0, eps=0.1, cep=_cep(2)),
                window=dict(wx=64, wy=64, wz=64, cx=0.0, cy=0.0, cz=0.0))


def c3():
    """Headline: float32, 512^3, dx = 1/12, two-octave single-cycle pulse,
    radial polarisation, f = 0.5, 1000 steps of dt = 1/24."""
    return dict(name="C3", n=(512, 512, 512), spacing=(1 / 12, 1 / 12, 1 / 12),
                precision="f32", dt=1.0 / 24.0, steps=1000,
                pulse=pulse(envelope="spectral", bandwidth=0.6, L=6.0, R0=16.0,
                            f_number=0.5, eps=0.1, polarization="radial",
                            cep=_cep(3)),
                window=dict(wx=64, wy=64, wz=64, cx=0.0, cy=0.0, cz=0.0))


def c4(ninst=64, seed=4):
    """Batched sweep: uneven cubes drawn from {128, 192, 256}^3, dx = 1/12,
    f ~ U[0.4, 2], CEP ~ U[0, 2 pi), GDD ~ U[-20, 20] fs^2; R0 chosen so the
    aperture fits in 80% of the half side; steps = round(R0 / dt)."""
    rng = np.random.default_rng(seed)
    d = 1.0 / 12.0
    dt = 0.5 * d
    out = []
    for i in range(ninst):
        n = int(rng.choice([128, 192, 256]))
        f = float(rng.uniform(0.4, 2.0))
        cep = float(rng.uniform(0.0, 2.0 * np.pi))
        gdd = float(rng.uniform(-20.0, 20.0)) / FS_PER_UNIT ** 2
        half = 0.5 * n * d
        # largest radius whose aperture (half-width 1/(2f) per unit radius
        # along the axis) stays within 80% of the transverse half side
        r_fit = 0.8 * half * np.sqrt(1.0 + 4.0 * f * f)
        R0 = float(min(16.0, r_fit))
        steps = int(round(R0 / dt))
        out.append(dict(n=(n, n, n), spacing=(d, d, d), precision="f32",
                        dt=dt, steps=steps,
                        pulse=pulse(envelope="spectral", bandwidth=1.0 / 3.0,
                                    L=6.0, R0=R0, f_number=f, eps=0.1,
                                    cep=cep, gdd=gdd),
                        window=dict(wx=64, wy=64, wz=64, cx=0.0, cy=0.0, cz=0.0)))
    return out


C5_RANGES = dict(f_number=(0.5, 2.0), cep=(0.0, 2.0 * np.pi),
                 gdd=(-20.0 / FS_PER_UNIT ** 2, 20.0 / FS_PER_UNIT ** 2),
                 tod=(-100.0 / FS_PER_UNIT ** 3, 100.0 / FS_PER_UNIT ** 3),
                 bandwidth=(0.2, 0.6), pol_angle=(0.0, np.pi),
                 ellipticity=(-1.0, 1.0), eps=(0.02, 0.3))
C5_KEYS = tuple(C5_RANGES)


def c5_params(n, seed):
    """n x 8 parameter draws (order of C5_KEYS), uniform in C5_RANGES."""
    rng = np.random.default_rng(seed)
    lo = np.array([C5_RANGES[k][0] for k in C5_KEYS])
    hi = np.array([C5_RANGES[k][1] for k in C5_KEYS])
    return lo + (hi - lo) * rng.uniform(size=(n, len(C5_KEYS)))


def c5_pulse(row):
    kw = dict(zip(C5_KEYS, (float(v) for v in row)))
    return pulse(envelope="spectral", L=6.0, R0=10.0, **kw)
