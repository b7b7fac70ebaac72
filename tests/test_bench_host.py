"""Host logic behind the bench line: the one-GPU guard, the rocprofv3
summaries (kernel names, copy-calibrated HBM bytes) and the rule that keeps
counter-measured traffic only while the pass kernels' sources are unchanged."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2010_00409_amd import profile_summary as ps  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]


def test_gemm_names_shorten_alike_demangled_or_not():
    dem = "void tf::fno::k_gemm<64, 128, 4, float, float, true>(tf::fno::GemmArgs)"
    man = "_ZN2tf3fno6k_gemmILi64ELi128ELi4EffLb1EEEvNS0_8GemmArgsE"
    assert ps._short(dem) == ps._short(man) == "k_gemm<64,128,4,float,float,true>"
    assert ps._short("_ZN2tf3fno6k_gemmILi32ELi64ELi2EfDF16bLb0EEEvNS0_8GemmArgsE") == \
        "k_gemm<32,64,2,float,bf16,false>"
    assert ps._short("void tf::k_z_fast<float, 512, 4, 8, 0, 8>(...)") == "k_z_fast"


def test_kernel_sources_follow_the_include_closure():
    names = [os.path.basename(p) for p in ps.kernel_sources()]
    assert names[0] == "fft_f32.hip"
    assert {"fft_passes.inc", "fft_core.h", "kernels.h"} <= set(names)
    assert "batch.hip" not in names and "fno.hip" not in names
    assert ps.source_hash() == ps.source_hash()


def _counter_csv(path, counter, rows):
    with open(path, "w") as f:
        f.write('"Kernel_Name","Grid_Size","Counter_Name","Counter_Value"\n')
        for name, grid, value in rows:
            f.write(f'"{name}",{grid},"{counter}",{value}\n')


def test_traffic_is_scaled_by_the_copy_calibration(tmp_path):
    # a 1 GiB copy that reads FETCH_SIZE at half its bytes and WRITE_SIZE at
    # its bytes, and a kernel moving 3 GiB in + 1 GiB out in counter units
    gib_kib = (1 << 30) / 1024
    fd, wd = tmp_path / "fetch", tmp_path / "write"
    fd.mkdir(), wd.mkdir()
    _counter_csv(fd / "a_counter_collection.csv", "FETCH_SIZE",
                 [("copy_kernel", 1 << 26, gib_kib / 2), ("copy_kernel", 1 << 10, 7.0),
                  ("k_z_fast<float>", 4096, 1.5 * gib_kib), ("k_z_fast<float>", 4096, 1.5 * gib_kib)])
    _counter_csv(wd / "a_counter_collection.csv", "WRITE_SIZE",
                 [("copy_kernel", 1 << 26, gib_kib), ("k_z_fast<float>", 4096, gib_kib)])
    text, rec, (fs, ws) = ps.traffic(str(fd), str(wd))
    assert fs == pytest.approx(2.0) and ws == pytest.approx(1.0)
    assert rec["k_z_fast"]["bytes_per_launch"] == pytest.approx(4 * (1 << 30))
    assert "k_z_fast" in text


def test_traffic_record_needs_the_current_kernel_sources(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    rec = {"k_z_fast": {"bytes_per_launch": 123.0, "source_sha256": ps.source_hash()}}
    (prof / "traffic.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "HERE", str(tmp_path))
    assert bench.traffic_record("k_z_fast") == 123.0
    rec["k_z_fast"]["source_sha256"] = "0" * 64
    (prof / "traffic.json").write_text(json.dumps(rec))
    assert bench.traffic_record("k_z_fast") is None
    assert bench.traffic_record("k_x_forward") is None


def test_pass_kernels_follow_the_plan():
    assert bench.pass_kernels((8, True, 7), 512)["z_step"] == "k_z_wave"
    assert bench.pass_kernels((8, True, 8), 512)["z_step"] == "k_z_wave"
    assert bench.pass_kernels((8, True, 7), 256)["z_step"] == "k_z_wave256"
    assert bench.pass_kernels((8, True, 7), 128)["z_step"] == "k_z_fast"
    assert bench.pass_kernels((8, True, 4), 256)["z_step"] == "k_z_fast"
    assert bench.pass_kernels((8, True, 6), 512)["z_step"] == "k_z_fast"
    k = bench.pass_kernels((8, False, 0), 512)
    assert (k["z_step"], k["y_forward"], k["x_inverse"]) == ("k_z", "k_col", "k_x_inverse")


def test_surrogate_bytes_grow_by_one_window_per_window():
    per = bench.surrogate_inference_bytes(2) - bench.surrogate_inference_bytes(1)
    assert per == bench.surrogate_inference_bytes(65) - bench.surrogate_inference_bytes(64)
    assert 300e6 < per < 450e6       # every tensor of one window written once and read once


def test_cpu_baseline_protocol_and_parity_on_a_small_layer():
    """The oracle leg of the bench on a small layer: warm-up + median of 3 at
    each size, cores and CPU model reported, and the parity object computed
    against the oracle's jump + cut-out (zero when the 'GPU' window is the
    oracle's own)."""
    import numpy as np
    from oracle import mapping, psatd, pulse
    from synthetic import configs
    p = configs.pulse(envelope="spectral", bandwidth=0.4, R0=4.0, L=3.0, f_number=0.5, nfreq=64)
    n, d = (24, 48, 48), 0.2
    grid = pulse.layer_grid(p, n, (d, d, d))
    E, B = pulse.init_fields(p, grid)
    E, B = psatd.step_fft(E, B, (d, d, d), 0.0, project_b_first=True)
    start = np.concatenate([E, B]).astype(np.float32)
    cfg = dict(spacing=(d, d, d), dt=0.1, pulse=p, grid=grid,
               window=dict(wx=8, wy=8, wz=8, cx=0.0, cy=0.0, cz=0.0))
    x = start.astype(np.float64)
    E, B = psatd.jump(x[:3], x[3:], (d, d, d), 40 * 0.1)
    geo = pulse.geometry(p)
    w = mapping.readout(np.concatenate([E, B]), grid, cfg["window"], 4.0, geo["R_min"], geo["R_max"])
    base, par = bench.cpu_baseline(start, cfg, 40, w, 4.0, mid=16, single=8)
    assert base["kind"] == "oracle" and base["cores"] >= 1 and base["value"] > 0
    assert "cpu_model" in base and base["single_thread_8"]["cores"] == 1
    assert base["at_16"]["s_per_step"] > 0 and "median of 3" in base["sample"]
    assert par["window_rel_l2"] <= 1e-15 and par["window_max_abs_over_peak"] <= 1e-15
    assert par["window_peak_abs"] > 0 and par["gate_rel_l2"] == pytest.approx(40 ** 0.5 * 1e-5)


def test_quoted_surrogate_reports_exist_and_state_their_transform():
    """The bench quotes the first committed training report it finds; each
    names its held-out error and the reports after the first are fallbacks.
    The padded-transform report states its period (the bench times inference
    at that period)."""
    found = [n for n in bench.SURROGATE_REPORTS if os.path.exists(os.path.join(bench.HERE, "profiles", n))]
    assert found and found[0] == bench.SURROGATE_REPORTS[0]
    for n in found:
        rep = json.load(open(os.path.join(bench.HERE, "profiles", n)))
        err = rep["test_rel_l2"]
        assert 0.0 < err["median"] <= err["mean"] <= err["max"]
        assert rep["n_test"] > 0 and rep["nbasis"] == 4
    first = json.load(open(os.path.join(bench.HERE, "profiles", found[0])))
    assert first["period"] > 64
