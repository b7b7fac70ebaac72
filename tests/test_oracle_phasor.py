"""Pins of the surrogate head's per-pulse weights (oracle.pulse.phasor_weights)
against the oracle's own pulse fields.  The solver is linear in the initial
field, so an identity of the initial fields carries over to the focal field.

* Two basis fields: the field of any carrier-envelope phase is the weighted
  sum of the same pulse at CEP = 0 and CEP = -sigma pi/2 (each un-normalised),
  everywhere in the pulse (the envelope is linear in exp(i sigma CEP)).
* Four basis fields: with d along y and along z, the same holds for any
  polarisation angle and ellipticity on the optical axis, where the direction
  factor R x (d x R) / |R x (d x R)| is linear in d."""
import math

import numpy as np
import pytest

from oracle import pulse
from synthetic import configs


def _fields(p, pts, unnormalised=True):
    g = pulse.geometry(p)
    E, B = pulse.fields_at(*pts, p, g)
    f = np.concatenate([E, B])
    if unnormalised and p["envelope"] == "spectral":
        f = f * pulse.spectral_norm(p)
    return f


def _points(p, n, on_axis, seed):
    rng = np.random.default_rng(seed)
    g = pulse.geometry(p)
    R = rng.uniform(g["R_min"], g["R_max"], n)
    a = 0.0 if on_axis else rng.uniform(0.0, g["alpha_max"], n)
    phi = rng.uniform(0, 2 * np.pi, n)
    return (-R * np.cos(a), R * np.sin(a) * np.cos(phi), R * np.sin(a) * np.sin(phi))


def _sigma(p):
    return 1.0 if p["envelope"] == "spectral" else -1.0


@pytest.mark.parametrize("envelope", ["spectral", "cos2", "gauss"])
def test_two_basis_weights_reproduce_any_cep_exactly(envelope):
    rng = np.random.default_rng(1)
    for trial in range(3):
        row = configs.c5_params(1, seed=10 + trial)[0]
        p = configs.c5_pulse(row)
        p = dict(p, envelope=envelope, L=4.0 if envelope != "spectral" else p["L"])
        pts = _points(p, 400, False, seed=trial)
        sig = _sigma(p)
        re = _fields(dict(p, cep=0.0), pts)
        im = _fields(dict(p, cep=-sig * math.pi / 2), pts)
        ref = _fields(p, pts, unnormalised=False)
        w = pulse.phasor_weights(p, 2)
        got = w[0] * re + w[1] * im
        assert np.abs(ref).max() > 1e-3
        assert np.abs(got - ref).max() <= 1e-11 * np.abs(ref).max(), (envelope, trial)


def test_four_basis_weights_reproduce_polarisation_on_axis():
    for trial in range(4):
        row = configs.c5_params(1, seed=20 + trial)[0]
        p = configs.c5_pulse(row)
        sig = _sigma(p)
        pts = _points(p, 200, True, seed=trial)
        basis = []
        for psi in (0.0, math.pi / 2):
            q = dict(p, pol_angle=psi, ellipticity=0.0)
            basis += [_fields(dict(q, cep=0.0), pts), _fields(dict(q, cep=-sig * math.pi / 2), pts)]
        ref = _fields(p, pts, unnormalised=False)
        w = pulse.phasor_weights(p, 4)
        got = sum(wk * b for wk, b in zip(w, basis))
        assert np.abs(ref).max() > 1e-3
        assert np.abs(got - ref).max() <= 1e-11 * np.abs(ref).max(), trial


def test_four_basis_weights_are_not_exact_off_axis():
    """Off the axis the normalisation of the direction factor depends on the
    polarisation angle; the four-basis head leaves that part to the network."""
    p = configs.c5_pulse(np.array([0.5, 1.0, 0.0, 0.0, 0.4, 0.7, 0.3, 0.1]))
    sig = _sigma(p)
    pts = _points(p, 400, False, seed=5)
    basis = []
    for psi in (0.0, math.pi / 2):
        q = dict(p, pol_angle=psi, ellipticity=0.0)
        basis += [_fields(dict(q, cep=0.0), pts), _fields(dict(q, cep=-sig * math.pi / 2), pts)]
    ref = _fields(p, pts, unnormalised=False)
    got = sum(wk * b for wk, b in zip(pulse.phasor_weights(p, 4), basis))
    assert np.abs(got - ref).max() > 1e-3 * np.abs(ref).max()
