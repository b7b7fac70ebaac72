"""Pulse on the focusing sphere and its mapping into the periodic layer
(oracle O3).

Test infrastructure only (see ``oracle/__init__``).

Closed forms followed:

* Sec. II.B: opening angle from the f-number, theta = arctan(1/(2f));
  flat-top transverse profile Eq. (5) with the rectangular window Eq. (6);
  cos^2 longitudinal profile Eq. (7); spherical pulse u(R) = (A/R) u_l(R-R0)
  u_ts(alpha), Eq. (8); amplitude A = sqrt(4 P0 / (c (1 - cos theta))),
  Eq. (9); E = u s0, B = u s1, Eqs. (10)-(11).
* Sec. III.B.1: Gaussian longitudinal envelope exp(-zeta^2 ln4/(n lambda)^2)
  with carrier sin(k zeta); Gaussian transverse profile exp(-alpha^2 /
  theta0^2); F(theta0) = int_0^pi sin(a) exp(-2 a^2/theta0^2) da.
* Sec. II.C: R_min,max = R0 -/+ L/2; D_min, Eq. (12); the layer
  x in [-R_min - D, -R_min]; the mapping T of Eq. (13), inverted here as a
  sum over the preimages x + n D of every layer node (superposition of
  replicas, the remark after Eq. (12)).

Readings:

* s1 = normalise(d x R), s0 = normalise(R x (d x R)) = component of d
  perpendicular to R; fields are 0 where d is parallel to R.
* alpha = angle from the -x axis = atan2(sqrt(y^2+z^2), -x).
* the first window of Eq. (5) is half-open, [0, theta - eps/2).
* layer nodes sum the contributions of all their preimages.
* x_min is shifted onto the node grid so the origin is a node.
* c = 1; fields in CGS form; A normalises the cycle-averaged power
  through the cap to P0.  Gaussian transverse: A = sqrt(4 P0 / F(theta0)).
* spectral envelope (not in the paper): g(zeta) = Re sum_m a_m exp(i phi_m)
  exp(-i w_m zeta) on M frequency samples; a(w) = G(w - w0) - G(w + w0),
  G(x) = exp(-(x/(delta w0))^2) (antisymmetrised so no DC radiates);
  phi = phase + pi/2 + GDD (w-w0)^2/2 + TOD (w-w0)^3/6; normalised so
  max |g| over zeta_j = j lambda/128 inside the window is 1.
* Gaussian and spectral envelopes are cut by the window [-L/2, L/2] of
  Eq. (6), L being the descriptor's support length.
* Elliptical polarisation: E = a1 u(phase) s0(d1) + a2 u(phase+pi/2) s0(d2)
  with d1 = (0, cos psi, sin psi), d2 = (0, -sin psi, cos psi),
  a1 = 1/sqrt(1+e^2), a2 = e/sqrt(1+e^2); radial polarisation is d = x.

A pulse descriptor is a dict with keys: envelope ('cos2'|'gauss'|'spectral'),
transverse ('flattop'|'gauss'), polarization ('linear'|'radial'),
wavelength, R0, L, ncycles, f_number, theta (>0 overrides f_number), eps,
P0, pol_angle, ellipticity, cep, gdd, tod, bandwidth, nfreq.
A grid is a dict nx, ny, nz, dx, dy, dz, x_min, y_min, z_min.
"""
import math

import numpy as np
import scipy.integrate

C_LIGHT = 1.0
SPECTRAL_HALF_WIDTH = 4.0   # samples span w0 (1 + delta x), |x| <= 4
NORM_SAMPLES_PER_WAVELENGTH = 128


def theta_of(p):
    """Opening angle, Sec. II.B: theta = arctan(1/(2 f))."""
    if p.get("theta", 0.0) > 0.0:
        return float(p["theta"])
    return math.atan(1.0 / (2.0 * p["f_number"]))


def F_gauss(theta0):
    """F(theta0) of Sec. III.B.1 by adaptive quadrature."""
    val, _ = scipy.integrate.quad(
        lambda a: math.sin(a) * math.exp(-2.0 * a * a / (theta0 * theta0)),
        0.0, math.pi, epsabs=0.0, epsrel=1e-13, limit=400)
    return val


def D_min(theta, R_min, R_max):
    """Smallest replica period without overlap, Eq. (12)."""
    return (-R_min * math.cos(theta)
            + math.sqrt(R_max * R_max - R_min * R_min * math.sin(theta) ** 2))


def geometry(p):
    """Host-side set-up: theta, amplitude, radii, D_min, angular support."""
    th = theta_of(p)
    L = float(p["L"])
    R0 = float(p["R0"])
    R_min, R_max = R0 - 0.5 * L, R0 + 0.5 * L
    if p["transverse"] == "flattop":
        A = math.sqrt(4.0 * p["P0"] / (C_LIGHT * (1.0 - math.cos(th))))
        alpha_max = th + 0.5 * p["eps"]
    else:
        A = math.sqrt(4.0 * p["P0"] / (C_LIGHT * F_gauss(th)))
        alpha_max = 0.5 * math.pi
    return dict(theta=th, A=A, R0=R0, L=L, R_min=R_min, R_max=R_max,
                D_min=D_min(th, R_min, R_max), alpha_max=alpha_max)


def u_ts(alpha, p, g):
    """Transverse profile: Eq. (5) (flat-top, first window half-open) or exp(-a^2/theta0^2)."""
    th = g["theta"]
    if p["transverse"] == "flattop":
        eps = p["eps"]
        lo, hi = th - 0.5 * eps, th + 0.5 * eps
        edge = np.cos(np.pi * (alpha - th + 0.5 * eps) / (2.0 * eps)) ** 2
        return np.where(alpha < lo, 1.0,
                        np.where(alpha <= hi, edge, 0.0))
    return np.where(alpha <= 0.5 * np.pi, np.exp(-(alpha * alpha) / (th * th)), 0.0)


def spectral_samples(p):
    """Frequency samples (w_m, a_m, chirp phase phi_m) of the sampled spectrum."""
    M = int(p["nfreq"])
    w0 = 2.0 * np.pi * C_LIGHT / p["wavelength"]
    dlt = p["bandwidth"]
    X = SPECTRAL_HALF_WIDTH
    x = -X + (np.arange(M) + 0.5) * (2.0 * X / M)
    w = w0 * (1.0 + dlt * x)
    keep = w > 0.0
    w = w[keep]
    a = np.exp(-((w - w0) / (dlt * w0)) ** 2) - np.exp(-((w + w0) / (dlt * w0)) ** 2)
    dw = w - w0
    phi = p["gdd"] * dw * dw / 2.0 + p["tod"] * dw * dw * dw / 6.0
    return w, a, phi


def g_spectral_raw(zeta, p, phase):
    """Unnormalised Re sum a_m exp(i (phase + pi/2 + phi_m - w_m zeta/c))."""
    w, a, phi = spectral_samples(p)
    zeta = np.asarray(zeta, dtype=np.float64)
    out = np.zeros(zeta.shape)
    for m in range(len(w)):
        out += a[m] * np.cos(phase + 0.5 * np.pi + phi[m] - w[m] * zeta / C_LIGHT)
    return out


def spectral_norm(p):
    """max |g| over zeta_j = j lambda/128 inside the window."""
    lam = p["wavelength"]
    h = lam / NORM_SAMPLES_PER_WAVELENGTH
    jmax = int(math.floor(0.5 * p["L"] / h))
    zs = np.arange(-jmax, jmax + 1) * h
    return float(np.abs(g_spectral_raw(zs, p, p["cep"])).max())


def u_l(zeta, p, phase, gnorm=None):
    """Longitudinal profile (carrier included) inside the window [-L/2, L/2]."""
    lam, L = p["wavelength"], p["L"]
    zeta = np.asarray(zeta, dtype=np.float64)
    inside = (zeta >= -0.5 * L) & (zeta <= 0.5 * L)
    env = p["envelope"]
    if env == "cos2":                                          # Eq. (7)
        val = np.sin(2.0 * np.pi * zeta / lam - phase) * np.cos(np.pi * zeta / L) ** 2
    elif env == "gauss":                                       # Sec. III.B.1
        n = p["ncycles"]
        val = (np.sin(2.0 * np.pi * zeta / lam - phase)
               * np.exp(-zeta * zeta * math.log(4.0) / (n * lam) ** 2))
    elif env == "spectral":                                    # sampled spectrum
        if gnorm is None:
            gnorm = spectral_norm(p)
        val = g_spectral_raw(zeta, p, phase) / gnorm
    else:
        raise ValueError(env)
    return np.where(inside, val, 0.0)


def pol_parts(p):
    """[(amplitude, d, phase offset)] of the polarisation model."""
    if p["polarization"] == "radial":
        return [(1.0, np.array([1.0, 0.0, 0.0]), 0.0)]
    psi, e = p.get("pol_angle", 0.0), p.get("ellipticity", 0.0)
    d1 = np.array([0.0, math.cos(psi), math.sin(psi)])
    d2 = np.array([0.0, -math.sin(psi), math.cos(psi)])
    n = math.sqrt(1.0 + e * e)
    parts = [(1.0 / n, d1, 0.0)]
    if e != 0.0:
        parts.append((e / n, d2, 0.5 * math.pi))
    return parts


def phasor_weights(p, nbasis):
    """Per-pulse weights of the surrogate's basis fields.

    Every envelope is u_l(zeta; phase) = Re[exp(i sigma phase) G(zeta)] with
    sigma = +1 for the spectral envelope (its phase enters as +phase) and -1
    for the cos^2 and Gaussian envelopes (sin(k zeta - phase), Eq. (7)); the
    spectral one is divided by gnorm, the others by 1.  The polarisation
    parts are (1/n) d1 at phase CEP and (e/n) d2 at CEP + pi/2, n = sqrt(1+e^2).
    Since the solver is linear, with z = exp(i sigma CEP):
      nbasis 1: [1]                                          (plain output)
      nbasis 2: [Re z, -Im z] / gnorm  -- weights of Re F, Im F, where F is the
                complex field of the same pulse at CEP = 0, gnorm = 1.  Exact.
      nbasis 4: [Re(z a), -Im(z a), Re(z b), -Im(z b)] / gnorm, the weights of
                Re F_y, Im F_y, Re F_z, Im F_z (d along y, z; CEP = 0; gnorm = 1)
                with a = (cos psi - i sigma e sin psi) / n, b = (sin psi + i sigma e cos psi) / n.
                Exact where the direction factor R x (d x R) / |R x (d x R)|
                is linear in d (on the optical axis); elsewhere its
                normalisation adds a polarisation-dependent correction.
    Radial polarisation: a = 1, b = 0."""
    if nbasis == 1:
        return np.ones(1)
    sig = 1.0 if p["envelope"] == "spectral" else -1.0
    gn = spectral_norm(p) if p["envelope"] == "spectral" else 1.0
    z = complex(math.cos(sig * p["cep"]), math.sin(sig * p["cep"]))
    if nbasis == 2:
        return np.array([z.real, -z.imag]) / gn
    if nbasis != 4:
        raise ValueError("nbasis must be 1, 2 or 4")
    if p["polarization"] == "radial":
        a, b = 1.0 + 0j, 0j
    else:
        psi, e = p.get("pol_angle", 0.0), p.get("ellipticity", 0.0)
        n = math.sqrt(1.0 + e * e)
        a = complex(math.cos(psi), -sig * e * math.sin(psi)) / n
        b = complex(math.sin(psi), sig * e * math.cos(psi)) / n
    za, zb = z * a, z * b
    return np.array([za.real, -za.imag, zb.real, -zb.imag]) / gn


def bump_phase(alpha, y, z, p):
    """Wavefront phase perturbation of Sec. III.B.3 at directions given by
    alpha (angle from -x) and the transverse position (y, z): a sum of
    Gaussian bumps exp(-|a - a_i|^2 / w_i^2) times amplitude_i over the
    angular position a = alpha (y, z) / rho (0 on the axis)."""
    bumps = p.get("bumps") or []
    rho = np.sqrt(y * y + z * z)
    safe = np.where(rho > 0.0, rho, 1.0)
    ay = np.where(rho > 0.0, alpha * y / safe, 0.0)
    az = np.where(rho > 0.0, alpha * z / safe, 0.0)
    ph = np.zeros(np.shape(alpha))
    for by, bz, amp, w in bumps:
        ph = ph + amp * np.exp(-((ay - by) ** 2 + (az - bz) ** 2) / (w * w))
    return ph


def fields_at(x, y, z, p, g, gnorm=None):
    """E, B (each a (3, ...) array) of the unmapped pulse at points.  A
    wavefront phase perturbation (p["bumps"]) adds to every polarisation
    part's carrier phase, as the CEP does."""
    x, y, z = (np.asarray(v, dtype=np.float64) for v in (x, y, z))
    x, y, z = np.broadcast_arrays(x, y, z)
    shape = x.shape
    x, y, z = x.ravel(), y.ravel(), z.ravel()
    E = np.zeros((3, x.size))
    B = np.zeros((3, x.size))
    R = np.sqrt(x * x + y * y + z * z)
    rho = np.sqrt(y * y + z * z)
    alpha = np.arctan2(rho, -x)                                # angle from -x
    zeta = R - g["R0"]
    support = (zeta >= -0.5 * g["L"]) & (zeta <= 0.5 * g["L"]) & (alpha <= g["alpha_max"])
    sel = np.nonzero(support)
    if len(sel[0]) == 0:
        return E.reshape((3,) + shape), B.reshape((3,) + shape)
    xs, ys, zs, Rs, al, ze = (v[sel] for v in (x, y, z, R, alpha, zeta))
    if p["envelope"] == "spectral" and gnorm is None:
        gnorm = spectral_norm(p)
    ts = u_ts(al, p, g)
    dph = bump_phase(al, ys, zs, p)
    for amp, d, ph in pol_parts(p):
        u = g["A"] / Rs * u_l(ze, p, p["cep"] + ph + dph, gnorm) * ts
        # s1 ~ d x R, s0 ~ R x (d x R)
        c1 = (d[1] * zs - d[2] * ys, d[2] * xs - d[0] * zs, d[0] * ys - d[1] * xs)
        n1 = np.sqrt(c1[0] * c1[0] + c1[1] * c1[1] + c1[2] * c1[2])
        c0 = (ys * c1[2] - zs * c1[1], zs * c1[0] - xs * c1[2], xs * c1[1] - ys * c1[0])
        ok = n1 > 0.0
        inv1 = np.where(ok, 1.0 / np.where(ok, n1, 1.0), 0.0)
        inv0 = np.where(ok, 1.0 / np.where(ok, n1 * Rs, 1.0), 0.0)
        for a in range(3):
            E[a][sel] += amp * u * c0[a] * inv0
            B[a][sel] += amp * u * c1[a] * inv1
    return E.reshape((3,) + shape), B.reshape((3,) + shape)


def layer_grid(p, n, spacing):
    """Periodic layer of Sec. II.C: D = nx dx, x_min = -R_min - D shifted onto
    the node grid so the origin is a node; y, z centred on the axis."""
    nx, ny, nz = n
    dx, dy, dz = spacing
    g = geometry(p)
    D = nx * dx
    i0 = math.floor((g["R_min"] + D) / dx + 0.5)
    return dict(nx=nx, ny=ny, nz=nz, dx=dx, dy=dy, dz=dz,
                x_min=-i0 * dx, y_min=-(ny // 2) * dy, z_min=-(nz // 2) * dz)


def preimage_range(grid, g):
    """Replica indices n that can bring some layer node into the support."""
    D = grid["nx"] * grid["dx"]
    xlo = grid["x_min"]
    xhi = grid["x_min"] + (grid["nx"] - 1) * grid["dx"]
    return (math.floor((-g["R_max"] - xhi) / D) - 1,
            math.ceil((g["R_max"] - xlo) / D) + 1)


def init_fields_at(p, grid, iz, iy, ix):
    """E, B at the layer nodes (iz, iy, ix): sum over preimages x + n D of
    the pulse (Eq. (13) inverted; preimages superpose).  With
    grid["replicate_yz"] the transverse periods Dy = ny dy, Dz = nz dz map
    the pulse too (duplication along y and z, Sec. II.C closing remarks):
    the sum also runs over y + m Dy, z + l Dz.  Returns two (3, npts) arrays."""
    g = geometry(p)
    gnorm = spectral_norm(p) if p["envelope"] == "spectral" else None
    D = grid["nx"] * grid["dx"]
    xt = grid["x_min"] + np.asarray(ix, dtype=np.float64) * grid["dx"]
    y = grid["y_min"] + np.asarray(iy, dtype=np.float64) * grid["dy"]
    z = grid["z_min"] + np.asarray(iz, dtype=np.float64) * grid["dz"]
    E = np.zeros((3,) + xt.shape)
    B = np.zeros((3,) + xt.shape)
    nlo, nhi = preimage_range(grid, g)
    shifts = [(0.0, 0.0)]
    if grid.get("replicate_yz"):
        Dy, Dz = grid["ny"] * grid["dy"], grid["nz"] * grid["dz"]
        R = g["R_max"]
        ms = range(math.floor((-R - y.max()) / Dy) - 1, math.ceil((R - y.min()) / Dy) + 2)
        ls = range(math.floor((-R - z.max()) / Dz) - 1, math.ceil((R - z.min()) / Dz) + 2)
        shifts = [(m * Dy, l * Dz) for l in ls for m in ms]
    for sy, sz in shifts:
        ys, zs = y + sy, z + sz
        if np.all(ys * ys + zs * zs > g["R_max"] ** 2):
            continue
        for n in range(nlo, nhi + 1):
            x = xt + n * D
            if np.all(np.abs(x) > g["R_max"]):
                continue
            e, b = fields_at(x, ys, zs, p, g, gnorm)
            E += e
            B += b
    return E, B


def init_fields(p, grid, chunk_z=8):
    """Full-grid initial E, B of shape (3, nz, ny, nx)."""
    nx, ny, nz = grid["nx"], grid["ny"], grid["nz"]
    E = np.zeros((3, nz, ny, nx))
    B = np.zeros((3, nz, ny, nx))
    iy, ix = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    for z0 in range(0, nz, chunk_z):
        zs = np.arange(z0, min(nz, z0 + chunk_z))
        IZ = np.broadcast_to(zs[:, None, None], (len(zs), ny, nx))
        IY = np.broadcast_to(iy[None], IZ.shape)
        IX = np.broadcast_to(ix[None], IZ.shape)
        e, b = init_fields_at(p, grid, IZ, IY, IX)
        E[:, z0:z0 + len(zs)] = e
        B[:, z0:z0 + len(zs)] = b
    return E, B
