"""The oracle against values the paper prints for its worked configurations
(fixture: tests/golden/paper_printed_values.json, each entry citing where the
paper prints it)."""
import json
import math
import os

import numpy as np
import pytest

from oracle import psatd, pulse
from synthetic import configs

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "paper_printed_values.json")
ENTRIES = {e["id"]: e for e in json.load(open(GOLDEN))["entries"]}


def _bytes_per_cell():
    """Bytes per node of the oracle's field state, from one oracle step."""
    rng = np.random.default_rng(0)
    E, B = rng.standard_normal((3, 8, 8, 8)), rng.standard_normal((3, 8, 8, 8))
    Eo, Bo = psatd.step_fft(E, B, (0.5, 0.5, 0.5), 0.1)
    return (Eo.nbytes + Bo.nbytes) // 8 ** 3


def test_opening_angle_of_f_number_03():
    e = ENTRIES["theta_f03"]
    th = pulse.theta_of(configs.pulse(f_number=e["inputs"]["f_number"]))
    assert th == pytest.approx(e["printed"], abs=e["abs_tol"])


def test_D_min_over_L_of_the_verification_case():
    """Reading: the aperture's smoothed edge widens the angular support from
    theta to theta + eps, and the printed 1.9 lies in the range Eq. (12)
    spans over it (1.70 at theta, 1.92 at theta + eps)."""
    e = ENTRIES["dmin_over_L_f03"]
    i = e["inputs"]
    th = pulse.theta_of(configs.pulse(f_number=i["f_number"]))
    R_min, R_max = i["R0"] - i["L"] / 2, i["R0"] + i["L"] / 2
    lo = pulse.D_min(th, R_min, R_max) / i["L"]
    hi = pulse.D_min(th + i["eps"], R_min, R_max) / i["L"]
    assert lo - e["abs_tol"] <= e["printed"] <= hi + e["abs_tol"]
    assert hi == pytest.approx(e["printed"], abs=e["abs_tol"])


def test_layer_against_direct_region_node_count():
    e = ENTRIES["direct_vs_layer_f03"]
    i = e["inputs"]
    d = i["spacing"]
    n_side = int(round(2 * i["half_width"] / d))
    nx = int(round(i["D"] / d))
    p = configs.pulse(R0=i["R0"], L=i["L"], f_number=i["f_number"], eps=i["eps"])
    g = pulse.layer_grid(p, (nx, n_side, n_side), (d, d, d))
    assert g["nx"] * g["dx"] == pytest.approx(i["D"])
    assert i["D"] >= pulse.geometry(p)["D_min"]           # the layer is a valid period
    ratio = n_side ** 3 / (g["nx"] * g["ny"] * g["nz"])
    assert e["range"][0] <= ratio <= e["range"][1]


def test_bytes_per_cell_of_the_double_precision_state():
    assert _bytes_per_cell() == ENTRIES["bytes_per_cell"]["printed"]


@pytest.mark.parametrize("key", ["grid_memory_D20", "grid_memory_D2"])
def test_memory_of_the_papers_grids(key):
    """(56 D/L) x 896 x 896 nodes at 28 points per wavelength: the layer spans
    D along x and the transverse extent 2 R0 along y and z; six float64
    components per node give the printed gigabytes (binary)."""
    e = ENTRIES[key]
    i = e["inputs"]
    d = 1.0 / i["points_per_wavelength"]
    n = (int(56 * i["D_over_L"]), 896, 896)
    g = pulse.layer_grid(configs.pulse(R0=i["R0"], L=i["L"]), n, (d, d, d))
    assert g["nx"] * g["dx"] == pytest.approx(i["D_over_L"] * i["L"])
    assert g["ny"] * g["dy"] == pytest.approx(2 * i["R0"])
    gib = g["nx"] * g["ny"] * g["nz"] * _bytes_per_cell() / 2 ** 30
    assert gib == pytest.approx(e["printed"], rel=e["rel_tol"])
    assert math.isfinite(gib)
