"""What the trained surrogate gains over the method without it, on MI355X.

A short training on solver-generated focal windows must (a) predict fresh
solver windows far better than the best parameter-blind predictor (the mean
training window) and (b) deliver a window in less time than the solver's
fastest exact route (pulse init + one jump step to t = R0 + cut-out).  The
fallback router must return the solver's windows bit for bit when the
tolerance excludes the surrogate."""
import numpy as np
import pytest
import torch

from paper_2010_00409_amd import surrogate as sg
from paper_2010_00409_amd import tfocus as tf
from synthetic import configs

pytestmark = pytest.mark.gpu

N_TRAIN, N_TEST, NB = 256, 16, 4


def _data(n, seed):
    rows = configs.c5_params(n, seed=seed)
    pulses = [configs.c5_pulse(r) for r in rows]
    y = torch.empty((n, 6, 64, 64, 64), dtype=torch.float32, device="cuda")
    sg.solver_windows(pulses, y)
    p = torch.from_numpy(sg.normalise(rows, configs.C5_RANGES, configs.C5_KEYS, NB).astype(np.float32)).cuda()
    return rows, pulses, p, sg.head_weights(pulses, NB), y


def test_trained_surrogate_beats_mean_field_and_solver_time():
    _, _, p_tr, w_tr, y_tr = _data(N_TRAIN, 101)
    _, pul_te, p_te, w_te, y_te = _data(N_TEST, 102)
    with tf.Surrogate(16, training=True, nbasis=NB) as s:
        s.set_params(sg.init_params(7, NB))
        hist = s.train(p_tr, y_tr, epochs=24, batch=16, lr=2e-3, w=w_tr, seed=7)
        flat = s.get_params()
    with tf.Surrogate(N_TEST, nbasis=NB) as inf:
        inf.set_params(flat)
        err = inf.eval(p_te, y_te, w=w_te)
        t_sur = sg.time_surrogate(inf, N_TEST, reps=5)
    # the best parameter-blind predictor: the mean training window (test-side reference)
    mean = y_tr.double().mean(dim=0, keepdim=True)
    d = (y_te.double() - mean).reshape(N_TEST, -1).norm(dim=1) / y_te.double().reshape(N_TEST, -1).norm(dim=1)
    mean_err = d.cpu().numpy()
    t_single, t_batch = sg.time_solver(pul_te[0], reps=2, batch=N_TEST)
    print(f"loss {hist[0]:.3f} -> {hist[-1]:.3f}; held-out {err.mean():.3f} vs mean field {mean_err.mean():.3f}; "
          f"surrogate {t_sur * 1e3:.3f} ms/window vs solver {t_batch * 1e3:.3f} ms/window")
    assert hist[-1] < 0.5 * hist[0]
    assert err.mean() < 0.5 * mean_err.mean()
    assert t_sur < t_batch


def test_fallback_returns_solver_windows_when_tolerance_excludes_surrogate():
    rows = configs.c5_params(3, seed=103)
    with tf.Surrogate(4, nbasis=NB) as inf:
        inf.set_params(sg.init_params(3, NB))
        ff = sg.FocalField(inf, validated_error=0.05, ranges=configs.C5_RANGES, keys=configs.C5_KEYS,
                           make_pulse=configs.c5_pulse)
        out = torch.zeros((3, 6, 64, 64, 64), dtype=torch.float32, device="cuda")
        used = ff(rows, tol=0.0, out=out)
        assert not used.any()
        ref = torch.empty_like(out)
        sg.solver_windows([configs.c5_pulse(r) for r in rows], ref)
        assert torch.equal(out, ref)
        out2 = torch.zeros_like(out)
        used2 = ff(rows, tol=0.1, out=out2)
        assert used2.all()
        w = sg.head_weights([configs.c5_pulse(r) for r in rows], NB)
        p = torch.from_numpy(sg.normalise(rows, configs.C5_RANGES, configs.C5_KEYS, NB).astype(np.float32)).cuda()
        direct = torch.empty_like(out)
        inf.forward(p, direct, w)
        assert torch.equal(out2, direct)
