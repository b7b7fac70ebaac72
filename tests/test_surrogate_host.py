"""Host logic of the surrogate workflow (no GPU): routing between the
surrogate and the solver fallback, and the parameter normalisation."""
import numpy as np

from paper_2010_00409_amd import surrogate
from synthetic import configs


def test_routing_uses_surrogate_only_within_tolerance_and_ranges():
    ff = surrogate.FocalField(None, 0.05, configs.C5_RANGES, configs.C5_KEYS, configs.c5_pulse)
    rows = configs.c5_params(6, seed=1)
    outside = rows[2].copy()
    outside[0] = configs.C5_RANGES["f_number"][1] + 0.1      # f-number beyond the training range
    rows = np.vstack([rows, outside])
    assert ff.route(rows, tol=0.1).tolist() == [True] * 6 + [False]
    assert not ff.route(rows, tol=0.01).any()                 # tolerance below the validated error
    assert not ff.route(rows, tol=0.0).any()                  # tolerance 0 forces the solver


def test_exactly_handled_parameters_are_hidden_from_the_network():
    rows = configs.c5_params(5, seed=3)
    i = configs.C5_KEYS.index("cep")
    p1 = surrogate.normalise(rows, configs.C5_RANGES, configs.C5_KEYS, 1)
    p4 = surrogate.normalise(rows, configs.C5_RANGES, configs.C5_KEYS, 4)
    assert np.all(p4[:, i] == 0) and np.all(p1[:, i] > 0)
    assert np.array_equal(np.delete(p1, i, axis=1), np.delete(p4, i, axis=1))


def test_normalise_maps_ranges_to_unit_interval():
    lo = np.array([configs.C5_RANGES[k][0] for k in configs.C5_KEYS])
    hi = np.array([configs.C5_RANGES[k][1] for k in configs.C5_KEYS])
    p = surrogate.normalise(np.vstack([lo, hi, 0.5 * (lo + hi)]), configs.C5_RANGES, configs.C5_KEYS)
    assert np.allclose(p, [[0] * 8, [1] * 8, [0.5] * 8])
    q = surrogate.normalise(configs.c5_params(100, seed=2), configs.C5_RANGES, configs.C5_KEYS)
    assert q.min() >= 0 and q.max() <= 1


def test_init_params_shapes_match_flat_layout():
    from paper_2010_00409_amd import tfocus as tf
    for nb in (1, 2, 4):
        P = surrogate.init_params(0, nb)
        assert tf.fno_flatten(P).size == tf.load().tf_fno_param_count(nb)
    assert np.all(P["b1"] == 0) and np.iscomplexobj(P["R2"])


def test_library_head_weights_equal_the_oracle():
    """tf_fno_phasor_weights (host code of the library) against the oracle's
    independent implementation, for both envelope phase conventions."""
    from oracle import pulse
    from paper_2010_00409_amd import tfocus as tf
    for seed in range(4):
        row = configs.c5_params(1, seed=seed)[0]
        for env in ("spectral", "cos2", "gauss"):
            p = dict(configs.c5_pulse(row), envelope=env, L=4.0)
            for nb in (1, 2, 4):
                a, b = tf.tf_fno_phasor_weights(p, nb), pulse.phasor_weights(p, nb)
                assert np.abs(a - b).max() <= 1e-14 * np.abs(b).max(), (seed, env, nb)
