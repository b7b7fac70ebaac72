"""Batched sweep of uneven grids and the autotuner, on the GPU.

The batch runs the same kernels as the single-grid solver with an instance
index in the launch grid, so every instance must equal the solver path bit
for bit; the captured graph must replay identically (with eager work in
between), and instances must match the oracle's exact jump."""
import os

import numpy as np
import pytest
import torch

from oracle import mapping, psatd, pulse
from paper_2010_00409_amd import tfocus as tf
from synthetic import configs

pytestmark = pytest.mark.gpu


def instances():
    """Seven instances on four grids (fast and generic kernel paths),
    different pulses and step counts (one with zero steps)."""
    rng = np.random.default_rng(7)
    out = []
    for n, d in ((64, 1 / 8), (64, 1 / 8), (64, 1 / 8), (48, 1 / 6), (48, 1 / 6), (96, 1 / 12), (32, 1 / 4)):
        f = float(rng.uniform(0.6, 1.5))
        p = configs.pulse(envelope="spectral", bandwidth=0.4, L=3.0, R0=3.0, f_number=f,
                          cep=float(rng.uniform(0, 6.28)), gdd=float(rng.uniform(-0.2, 0.2)), nfreq=64)
        g = pulse.layer_grid(p, (n, n, n), (d, d, d))
        out.append((g, p, 0.5 * d))
    nsteps = [12, 5, 0, 9, 9, 7, 4]
    return out, nsteps


WIN = dict(wx=16, wy=16, wz=16, cx=0.0, cy=0.0, cz=0.0)


def solver_reference(g, p, nsteps, dt):
    with tf.Solver(g, "f32") as s:
        s.set_pulse(p)
        s.advance(nsteps, dt)
        st = np.empty(s.shape, np.float32)
        s.get_fields(st)
        w = np.empty((6, WIN["wz"], WIN["wy"], WIN["wx"]), np.float32)
        s.read_focal(WIN, w)
    return st, w


def test_batch_equals_solver_path_and_graph_replays():
    inst, nsteps = instances()
    grids = [i[0] for i in inst]
    pulses = [i[1] for i in inst]
    dts = [i[2] for i in inst]
    n = len(inst)
    wsz = (6, WIN["wz"], WIN["wy"], WIN["wx"])
    outs = []
    with tf.Batch(grids, pulses, "f32") as b:
        for use_graph in (True, True, False, True):
            dst = torch.zeros((n,) + wsz, dtype=torch.float32, device="cuda")
            b.run(nsteps, dts, WIN, dst, use_graph=use_graph)
            torch.cuda.synchronize()
            junk = torch.randn(1 << 20, device="cuda").sum()     # eager work between replays
            torch.cuda.synchronize()
            del junk
            outs.append(dst.cpu().numpy())
        states = []
        for i in range(n):
            g = grids[i]
            st = np.empty((6, g["nz"], g["ny"], g["nx"]), np.float32)
            b.get_fields(i, st)
            states.append(st)
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])
    for i in range(n):
        ref_state, ref_win = solver_reference(grids[i], pulses[i], nsteps[i], dts[i])
        assert np.array_equal(states[i], ref_state), i
        assert np.array_equal(outs[0][i], ref_win), i
    assert np.abs(outs[0]).max() > 0


def test_batch_instances_match_oracle_jump():
    inst, nsteps = instances()
    for i in (0, 3, 5):
        g, p, dt = inst[i]
        with tf.Batch([g], [p], "f32") as b:
            dst = torch.zeros((1, 6, 16, 16, 16), dtype=torch.float32, device="cuda")
            b.run([nsteps[i]], [dt], WIN, dst)
            st = np.empty((6, g["nz"], g["ny"], g["nx"]), np.float32)
            b.get_fields(0, st)
            w = dst.cpu().numpy()[0]
        E, B = pulse.init_fields(p, g)
        E, B = psatd.step_fft(E, B, (g["dz"], g["dy"], g["dx"]), 0.0, project_b_first=True)
        E, B = psatd.jump(E, B, (g["dz"], g["dy"], g["dx"]), nsteps[i] * dt)
        ref = np.concatenate([E, B])
        err = np.linalg.norm(st - ref) / np.linalg.norm(ref)
        assert err < 2e-4, (i, err)
        geo = pulse.geometry(p)
        wref = mapping.readout(ref, g, WIN, 0.0 + nsteps[i] * dt, geo["R_min"], geo["R_max"])
        assert np.linalg.norm(w - wref) <= 2e-4 * max(np.linalg.norm(wref), 1e-30)


def test_batch_rejects_bad_arguments():
    inst, nsteps = instances()
    g, p, dt = inst[0]
    with tf.Batch([g], [p], "f32") as b:
        dst = torch.zeros((1, 6, 16, 16, 16), dtype=torch.float32, device="cuda")
        with pytest.raises(tf.TfError):
            b.run([-1], [dt], WIN, dst)
        with pytest.raises(tf.TfError):
            b.run([1], [dt], dict(WIN, wy=1000), torch.zeros((1, 6, 16, 1000, 16), device="cuda"))
    bad = dict(g, nx=g["nx"], dx=0.001)          # D = nx dx <= L
    with pytest.raises(tf.TfError) as ei:
        tf.Batch([bad], [p], "f32")
    assert ei.value.status == tf.TF_EDOMAIN


def test_tuner_writes_plans_that_keep_parity(tmp_path):
    plan = str(tmp_path / "plans.txt")
    best = tf.tf_tune([32, 64], "f32", plan)
    assert len(best) == 2 and all(b > 0 for b in best)
    lines = [l.split() for l in open(plan) if not l.startswith("#")]
    assert len(lines) == 2 and {l[2] for l in lines} == {"32", "64"}
    tf.tf_set_plan_file(plan)
    try:
        g = configs.cube_grid(64, 0.25)
        x = np.random.default_rng(9).standard_normal((6, 64, 64, 64)).astype(np.float32)
        with tf.Solver(g, "f32") as s:
            s.set_fields(x)
            s.advance(1, 0.3)
            out = np.empty(s.shape, np.float32)
            s.get_fields(out)
        Eo, Bo = psatd.step_fft(x[:3].astype(np.float64), x[3:].astype(np.float64), (0.25,) * 3, 0.3)
        ref = np.concatenate([Eo, Bo])
        assert np.linalg.norm(out - ref) / np.linalg.norm(ref) <= 1e-5
    finally:
        tf.tf_set_plan_file(None)
