"""Benchmark of the headline workload on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-surrogate]
    python bench.py --workload c4          # batched sweep of 64 uneven grids
    python bench.py --workload surrogate   # the surrogate section alone

Workload (C3): a 512^3 float32 periodic layer, dx = lambda/12, a two-octave
single-cycle spectral pulse (f = 0.5, radial polarisation) put on the
focusing sphere and mapped into the layer, 1000 spectral steps of
dt = lambda/24, then the 64^3 focal window read through the cut-out.  One
bench "step" is one such run (init + 1000 steps + readout); W runs are
untimed, K runs are timed between device synchronisations.  Inputs are
synthetic and generated on the device by the library.

Printed: one JSON line with the whole-run throughput in cell-updates/s, the
roofline of the dominant kernel (algorithmic bytes over its mean launch time
from HIP events recorded around every launch in the timed region, with the
counter-measured bytes of the same kernel when they were taken on the
current sources), the CPU oracle timed on this host on a bounded sample, and
the surrogate section: time to the 64^3 focal window of the learned
surrogate (one graph replay) and of the solver's exact route (init + one
step of dt = R0 + cut-out), measured here, and the held-out error of the
committed training report.
"""
import argparse
import json
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

PEAK_HBM_GBS = 8000.0
METRIC = "PSATD cell-updates/s + HBM GB/s at 512^3 FP32; surrogate speedup at 1e-2 err"
PASS_BYTES_PER_CELL = {"f32": 48, "f64": 96}   # read + write of six components
# kernel behind each pass of the float32 512^3 step (rocprofv3 short names)
PASS_KERNEL = {"x_forward": "k_x_forward", "y_forward": "k_col_fast", "z_step": "k_z_fast",
               "y_inverse": "k_col_fast", "x_inverse": "k_x_inverse"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2, help="timed runs")
    ap.add_argument("--warmup", type=int, default=1, help="untimed runs")
    ap.add_argument("--psatd-steps", type=int, default=None, help="override steps per run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", default="c3", choices=["c3", "c2", "c4", "surrogate"])
    ap.add_argument("--no-surrogate", action="store_true", help="skip the surrogate timing on c3/c2")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration)")
    return ap.parse_args()


def traffic_record(kernel):
    """HBM bytes per launch measured by rocprofv3 counters for this kernel,
    if recorded against the current kernel source (else None)."""
    path = os.path.join(HERE, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path)).get(PASS_KERNEL.get(kernel, kernel))
    if not rec:
        return None
    from paper_2010_00409_amd.profile_summary import source_hash
    if rec.get("source_sha256") != source_hash():
        return None
    return rec.get("bytes_per_launch")


def cpu_baseline(n, seed=3):
    """The oracle's spectral step (float64 real FFTs, Eqs. (3)-(4)) on one
    n^3 state with random fields: a bounded sample of the workload's step."""
    import numpy as np
    from oracle import psatd
    rng = np.random.default_rng(seed)
    E = rng.standard_normal((3, n, n, n))
    B = rng.standard_normal((3, n, n, n))
    d = 1.0 / 12.0
    cores = psatd._workers()
    t0 = time.perf_counter()
    psatd.step_fft(E, B, (d, d, d), 1.0 / 24.0, workers=cores)
    dt = time.perf_counter() - t0
    return {"value": n ** 3 / dt, "unit": "cell-updates/s", "cores": cores, "kind": "oracle",
            "sample": f"one float64 oracle step (scipy rfftn -> Eqs. (3)-(4) -> irfftn, "
                      f"{cores} workers) of a {n}^3 six-component state: {dt:.2f} s"}


# surrogate training report whose held-out error the bench quotes (written by
# python -m paper_2010_00409_amd.surrogate on MI355X; the weights themselves
# are not kept, and inference time does not depend on their values)
SURROGATE_REPORTS = ("surrogate_k4_head_4000x230_batch4.json", "surrogate_k4_head_4000x320_batch8.json", "surrogate_k4_head_4000x400.json", "surrogate_k4_head_4000x340.json", "surrogate_k4_head_4000x200.json",
                     "surrogate_k4_head_4000x140.json", "surrogate_k4_head_4000x60.json")


def surrogate_inference_bytes(batch):
    """Algorithmic HBM bytes of one fused inference pass over `batch`
    windows: every tensor the pass writes once and reads once, plus the
    bf16 spectral weights once per pass."""
    N, C, LINE = 64, 32, 12 * 32
    x1, x2, x3 = N * N * 2 * LINE, 24 * N * 2 * LINE, 24 * 2 * 24 * LINE
    node, out = N ** 3 * C, 6 * N ** 3
    per_layer = 2 * x1 + 4 * x2 + 4 * x3    # y, z contractions, mixing, z, y expansions
    lines = [x1 + node + x1,            # layer 0: U1 in, v1 out, X1 out (v0 recomputed)
             x1 + node + node + x1,     # layer 1
             x1 + node + out]           # layer 2 + projection
    per_window = 4 * (x1 + 3 * per_layer + sum(lines))
    weights = 3 * 6912 * 64 * 64 * 2
    return per_window * batch + weights


def surrogate_section(reps=20, batch=64):
    """Time-to-focal-field of the surrogate (one graph replay per batch) and
    of the solver (one exact jump step per window), measured live."""
    import torch
    from paper_2010_00409_amd import surrogate as sg
    from paper_2010_00409_amd import tfocus as tf
    from synthetic import configs

    sur = tf.Surrogate(batch, nbasis=4)
    sur.set_params(sg.init_params(0, 4))
    t_b = sg.time_surrogate(sur, batch, reps=reps)
    t_1 = sg.time_surrogate(sur, 1, reps=reps)
    sur.close()
    pulse = configs.c5_pulse(configs.c5_params(1, seed=configs.ROOT_SEED)[0])
    t_sol1, t_solb = sg.time_solver(pulse, reps=3, batch=batch)
    alg = surrogate_inference_bytes(batch)
    achieved = alg / (t_b * batch) / 1e9
    rep, src = None, None
    for name in SURROGATE_REPORTS:
        path = os.path.join(HERE, "profiles", name)
        if os.path.exists(path):
            rep, src = json.load(open(path)), "profiles/" + name
            break
    err = rep["test_rel_l2"] if rep else None
    return {
        "s_per_window": {"batch1": t_1, f"batch{batch}": t_b},
        "solver_s_per_window": {"single": t_sol1, f"batch{batch}": t_solb},
        "speedup": {"batch1_vs_single": t_sol1 / t_1, f"batch{batch}": t_solb / t_b},
        "heldout_rel_l2": err, "heldout_source": src,
        "meets_1e-2": (err["mean"] <= 1e-2) if err else None,
        "roofline": {"bound": "hbm", "kernel": "fused inference pass", "achieved": achieved,
                     "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS,
                     "alg_bytes_per_launch": alg},
        "workload": ("C5: 3-layer FNO (width 32, 12 modes/axis, four-basis head) -> 6 x 64^3 focal window; "
                     "solver: 96x256x256 layer, dx = lambda/12, one exact step to t = R0, cut-out"),
    }


def bench_c4(args):
    """Batched sweep (C4): 64 instances on uneven grids {128, 192, 256}^3,
    each init + its own steps to the focus + 64^3 cut-out, all in one
    captured graph per sweep.  One bench step = one sweep."""
    import torch
    from paper_2010_00409_amd import tfocus as tf
    from synthetic import configs

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    insts = configs.c4()
    grids = [tf.tf_layer_grid(c["pulse"], c["n"], c["spacing"]) for c in insts]
    pulses = [c["pulse"] for c in insts]
    nsteps = [c["steps"] for c in insts]
    dts = [c["dt"] for c in insts]
    win = insts[0]["window"]
    dst = torch.empty((len(insts), 6, win["wz"], win["wy"], win["wx"]), dtype=torch.float32, device="cuda")
    updates = sum(c["n"][0] ** 3 * c["steps"] for c in insts)
    with tf.Batch(grids, pulses, "f32", stream) as b:
        for _ in range(args.warmup):
            b.run(nsteps, dts, win, dst)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            b.run(nsteps, dts, win, dst)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
    el = t1 - t0
    sizes = {}
    for c in insts:
        sizes[c["n"][0]] = sizes.get(c["n"][0], 0) + 1
    print(json.dumps({
        "metric": "batched sweep cell-updates/s (64 uneven grids, one graph per sweep)",
        "value": updates * args.steps / el, "unit": "cell-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "C4: 64 instances, sizes " + json.dumps(sizes) +
                   ", dx = lambda/12, f ~ U[0.4, 2], CEP, GDD; steps to the focus; 64^3 cut-out",
                   "cell_updates_per_sweep": updates, "total_steps": sum(nsteps)},
        "focal_peak_abs": float(dst.abs().max().item()),
    }), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.workload == "c4":
        bench_c4(args)
        return
    if args.workload == "surrogate":
        sec = surrogate_section(reps=max(args.steps, 1))
        t = sec["s_per_window"]["batch64"]
        print(json.dumps({
            "metric": "surrogate focal windows/s (one graph replay per 64 windows)",
            "value": 1.0 / t, "unit": "windows/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": t * 64 * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "bf16", "data": "synthetic", "config": {"workload": sec["workload"]},
            "roofline": sec["roofline"], "surrogate": sec}), flush=True)
        return
    import torch
    from paper_2010_00409_amd import tfocus as tf
    from synthetic import configs

    cfg = configs.c3() if args.workload == "c3" else configs.c2()
    n = cfg["n"]
    steps = args.psatd_steps or cfg["steps"]
    prec = cfg["precision"]
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    grid = tf.tf_layer_grid(cfg["pulse"], n, cfg["spacing"])
    win = cfg["window"]
    dtype = torch.float32 if prec == "f32" else torch.float64
    out = torch.empty((6, win["wz"], win["wy"], win["wx"]), dtype=dtype, device="cuda")
    cells = n[0] * n[1] * n[2]

    # the focal window is read when the pulse centre reaches the focus
    focus_step = min(steps, int(round(cfg["pulse"]["R0"] / cfg["dt"])))

    with tf.Solver(grid, prec, stream) as s:
        def run():
            s.set_pulse(cfg["pulse"])
            s.advance(focus_step, cfg["dt"])
            s.read_focal(win, out)
            s.advance(steps - focus_step, cfg["dt"])

        for _ in range(args.warmup):
            run()
        torch.cuda.synchronize()
        s.profile(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            run()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        prof = s.profile_read()
        s.profile(False)
        peak_field = float(out.abs().max().item())

    if args.calibrate_copy:
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    elapsed = t1 - t0
    cell_updates = cells * steps * args.steps
    value = cell_updates / elapsed
    passes = {k: v for k, v in prof.items() if v[1] > 0}
    step_passes = ("x_forward", "y_forward", "z_step", "y_inverse", "x_inverse")
    dom = max(step_passes, key=lambda k: passes.get(k, (0.0, 0))[0])
    dom_ms, dom_n = passes[dom]
    per_launch_s = dom_ms / dom_n / 1e3
    alg_bytes = PASS_BYTES_PER_CELL[prec] * cells
    achieved = alg_bytes / per_launch_s / 1e9
    traffic = traffic_record(dom)
    step_ms = sum(passes[k][0] for k in step_passes) / (steps * args.steps)
    hbm_gbs = PASS_BYTES_PER_CELL[prec] * len(step_passes) * cells / (step_ms / 1e3) / 1e9

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": prec,
        "data": "synthetic",
        "config": {
            "workload": (f"{cfg['name']}: {n[0]}^3 {prec} periodic layer, dx = lambda/{round(1 / cfg['spacing'][0])}, "
                         f"spectral pulse mapped into the layer, {steps} steps of dt = {cfg['dt']:.6g}, "
                         f"64^3 focal window read at the focus (step {focus_step}); "
                         f"one bench step = init + {steps} steps + readout"),
            "grid": list(n), "psatd_steps_per_run": steps, "precision": prec,
            "twiddles_and_phases": "float64-built",
        },
        "hbm_gbs_pass_model": hbm_gbs,
        "ms_per_psatd_step": step_ms,
        "passes_ms_per_launch": {k: v[0] / v[1] for k, v in passes.items()},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS,
                     "traffic": traffic, "alg_bytes_per_launch": alg_bytes},
        "focal_peak_abs": peak_field,
    }
    if not args.no_surrogate:
        line["surrogate"] = surrogate_section()
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(n[0])
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
