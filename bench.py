"""Benchmark of the headline workload on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-surrogate]
    python bench.py --workload c4          # batched sweep of 64 uneven grids
    python bench.py --workload surrogate   # the surrogate section alone
    python bench.py --workload verify|duplicate|paraxial|flattop|perturbed
                                           # the paper's verification and focusing examples

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


def pass_kernels(plan, nz):
    """Kernel (rocprofv3 short name) behind each pass of a step under a kernel
    plan (row_block, fast, zvariant, ...) with nz-point z columns."""
    _, fast, zv = plan[:3]
    if not fast:
        z, col = "k_z", "k_col"
    else:
        waves = {512: "k_z_wave", 256: "k_z_wave256"}
        z, col = (waves[nz] if zv >= 7 and nz in waves else "k_z_fast"), "k_col_fast"
    return {"x_forward": "k_x_forward", "y_forward": col, "z_step": z, "y_inverse": col,
            "x_inverse": "k_x_inverse"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2, help="timed runs")
    ap.add_argument("--warmup", type=int, default=1, help="untimed runs")
    ap.add_argument("--psatd-steps", type=int, default=None, help="override steps per run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", default="c3", choices=["c3", "c2", "c4", "surrogate", "verify", "paraxial",
                                                         "flattop", "perturbed", "duplicate"])
    ap.add_argument("--no-surrogate", action="store_true", help="skip the surrogate timing on c3/c2")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration)")
    return ap.parse_args()


def traffic_record(kernel):
    """HBM bytes per launch measured by rocprofv3 counters for this kernel
    (short name), if recorded against the current kernel source (else None)."""
    path = os.path.join(HERE, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path)).get(kernel)
    if not rec:
        return None
    from paper_2010_00409_amd.profile_summary import source_hash
    if rec.get("source_sha256") != source_hash():
        return None
    return rec.get("bytes_per_launch")


def cpu_model():
    """CPU model string of this host (/proc/cpuinfo), or None."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.lower().startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _median_step(fn, reps=3):
    """Median wall time of reps calls after one untimed warm-up call (which
    also builds the FFT plans); returns (seconds, last result)."""
    out = fn()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        out = fn()
        ts.append(time.perf_counter() - t0)
    return sorted(ts)[len(ts) // 2], out


def cpu_baseline(start, cfg, focus_step, window_gpu, t_focus, mid=256, single=128):
    """The oracle (float64 scipy rfftn -> Eqs. (3)-(4) -> irfftn) timed on
    this host: median of 3 steps after a warm-up at the workload's size (the
    exact jump from the GPU's start state to the focus, a step like any
    other) and at 256^3 (random fields) with every host core, and
    single-threaded at 128^3 for ns per cell next to the paper's CPU figure.
    The 512^3 jump also gives the parity of the GPU's focal window against the
    float64 oracle (relative L2 and max |error| / peak, Sec. III.A)."""
    import numpy as np
    from oracle import mapping, psatd, pulse
    cores = psatd._workers()
    geo = pulse.geometry(cfg["pulse"])
    n = start.shape[1:]
    sp = tuple(cfg["spacing"][::-1])
    x = start.astype(np.float64)
    T = focus_step * cfg["dt"]
    t_big, (E, B) = _median_step(lambda: psatd.jump(x[:3], x[3:], sp, T, workers=cores))
    ref = np.concatenate([E, B])
    del E, B, x
    wref = mapping.readout(ref, cfg["grid"], cfg["window"], t_focus, geo["R_min"], geo["R_max"])
    del ref
    wgpu = window_gpu.astype(np.float64)
    peak = float(np.abs(wref).max())
    parity = {"against": f"float64 oracle: one exact jump of {focus_step} dt from the GPU state after the "
                         "one-time removal of longitudinal B (a dt = 0 step of tf_set_pulse's init), then the cut-out",
              "window_rel_l2": float(np.linalg.norm(wgpu - wref) / np.linalg.norm(wref)),
              "window_max_abs_over_peak": float(np.abs(wgpu - wref).max() / peak),
              "window_peak_abs": peak,
              "gate_rel_l2": math.sqrt(focus_step) * 1e-5}
    rng = np.random.default_rng(3)
    m = mid
    y = rng.standard_normal((6, m, m, m))
    d = cfg["spacing"][0]
    t_mid, _ = _median_step(lambda: psatd.step_fft(y[:3], y[3:], (d, d, d), cfg["dt"], workers=cores))
    del y
    k = single
    z = rng.standard_normal((6, k, k, k))
    t_one, _ = _median_step(lambda: psatd.step_fft(z[:3], z[3:], (d, d, d), cfg["dt"], workers=1))
    cells = n[0] * n[1] * n[2]
    base = {
        "value": cells / t_big, "unit": "cell-updates/s", "cores": cores, "kind": "oracle",
        "cpu_model": cpu_model(),
        "sample": (f"median of 3 float64 oracle steps after one warm-up at {n[2]}x{n[1]}x{n[0]} "
                   f"({cores} scipy workers; each the exact jump to the focus): {t_big:.2f} s per step"),
        f"at_{m}": {"cell_updates_per_s": m ** 3 / t_mid, "s_per_step": t_mid, "cores": cores,
                   "sample": "median of 3 steps after one warm-up, random fields"},
        f"single_thread_{k}": {"ns_per_cell": t_one / k ** 3 * 1e9, "s_per_step": t_one, "cores": 1,
                              "paper_context": "230 ns per cell per iteration, float64, single thread, "
                                               "Xeon Gold 6154 with MKL (Sec. III.A; other hardware, context only)"},
    }
    return base, parity


# surrogate training reports whose held-out error the bench quotes, first
# found wins (written by python -m paper_2010_00409_amd.surrogate on MI355X;
# the weights themselves are not kept, and inference time does not depend on
# their values): the spectral path on an 80-periodic zero-padded domain, then
# the plain 64-periodic one
SURROGATE_REPORTS = ("surrogate_k4_head_p80_4000x370_batch16.json", "surrogate_k4_head_4000x230_batch4.json")


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

    rep, src = None, None
    for name in SURROGATE_REPORTS:
        path = os.path.join(HERE, "profiles", name)
        if os.path.exists(path):
            rep, src = json.load(open(path)), "profiles/" + name
            break
    err = rep["test_rel_l2"] if rep else None
    period = rep.get("period", 64) if rep else 64
    sur = tf.Surrogate(batch, nbasis=4, period=period)
    sur.set_params(sg.init_params(0, 4))
    t_b = sg.time_surrogate(sur, batch, reps=reps)
    t_1 = sg.time_surrogate(sur, 1, reps=reps)
    sur.close()
    pulse = configs.c5_pulse(configs.c5_params(1, seed=configs.ROOT_SEED)[0])
    t_sol1, t_solb = sg.time_solver(pulse, reps=3, batch=batch)
    alg = surrogate_inference_bytes(batch)
    achieved = alg / (t_b * batch) / 1e9
    return {
        "s_per_window": {"batch1": t_1, f"batch{batch}": t_b},
        "solver_s_per_window": {"single": t_sol1, f"batch{batch}": t_solb},
        "speedup": {"batch1_vs_single": t_sol1 / t_1, f"batch{batch}": t_solb / t_b},
        "heldout_rel_l2": err, "heldout_source": src, "spectral_period": period,
        "meets_1e-2": (err["mean"] <= 1e-2) if err else None,
        "roofline": {"bound": "hbm", "kernel": "fused inference pass", "achieved": achieved,
                     "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS,
                     "alg_bytes_per_launch": alg},
        "workload": (f"C5: 3-layer FNO (width 32, 12 modes/axis of a {period}-periodic transform, four-basis head) "
                     "-> 6 x 64^3 focal window; "
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


def bench_verify(args):
    """The method against direct computation (Sec. III.A, Fig. 4a): a 512^3
    direct cube and periodic layers of D/L = 1.33 ... 8 at 12 points per
    wavelength, f = 0.3, L = 2, eps = 0.1, R0 = 16, one exact step to the
    focus; focal error (max |diff| / peak) and the time and memory the layers
    save, in float32 and float64."""
    import torch
    from paper_2010_00409_amd import verify

    torch.cuda.set_device(0)
    if args.workload == "duplicate":
        dup = verify.transverse_duplication((64, 96, 128, 192, 256), reps=max(args.steps, 1))
        at = [r for r in dup["boxes"] if r["n_t"] == 128][0]
        print(json.dumps({
            "metric": "transverse duplication: focal error (max |diff| / peak) of a 128^2 transverse box",
            "value": at["max_err_over_peak"], "unit": "fraction of peak", "n_gpus": 1, "steps": args.steps,
            "warmup": 1, "ms_per_step": at["seconds"] * 1e3, "higher_is_better": False, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "Sec. II.C closing remarks: Sec. III.A pulse, layer of 128 nodes (D/L = 5.33) "
                                   "at dx = lambda/12, transverse boxes replicated along y and z against the "
                                   "512^2 layer, one step to the focus, 64^3 window"},
            "sweep": dup}), flush=True)
        return
    layers = (32, 48, 64, 96, 128, 192)           # D/L = 1.33 (overlapping) ... 8
    res = {prec: verify.mapped_vs_direct(layers, precision=prec, reps=max(args.steps, 1))
           for prec in ("f32", "f64")}
    at4 = [r for r in res["f32"]["layers"] if r["nx"] == 96][0]
    print(json.dumps({
        "metric": "mapped layer vs direct cube: focal error (max |diff| / peak) at D/L = 4, f = 0.3",
        "value": at4["max_err_over_peak"], "unit": "fraction of peak", "n_gpus": 1, "steps": args.steps,
        "warmup": 1, "ms_per_step": at4["seconds"] * 1e3, "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "Sec. III.A verification: 512^3 direct cube vs periodic layers nx x 512 x 512, "
                               "dx = lambda/12, one step of dt = R0 = 16, 64^3 focal window through the cut-out"},
        "paper_context": "0.9% at D_min/L ~ 1.9 and under 0.1% at D/L ~ 3.5 (12 points/lambda); 0.12% at "
                         "D/L = 3.5 with time cut almost 6x (48 points/lambda); MVS-10P CPU node, float64",
        "sweep": {prec: {"D_min_over_L": r["D_min_over_L"], "direct_seconds": r["direct_seconds"],
                         "direct_bytes": r["direct_bytes"], "layers": r["layers"]} for prec, r in res.items()},
    }), flush=True)


def bench_examples(args):
    """The paper's focusing examples: the Gaussian beam of Sec. III.B.1 (peak
    intensity at the focus against the paraxial I0 = 2 P0 / (pi w0^2) for
    f = 0.25 ... 2, 512^3 nodes over 40 lambda) or the flat-top pulse of
    Sec. III.B.2 (peak intensity and where it is reached against f, D = 2 L
    on 128 x 1024 x 1024 nodes), or the same pulse at f = 1 under random
    wavefront perturbations (Sec. III.B.3)."""
    import torch
    from paper_2010_00409_amd import verify

    torch.cuda.set_device(0)
    fs = (0.25, 0.35, 0.5, 0.7, 1.0, 1.4, 2.0)
    t0 = time.perf_counter()
    if args.workload == "paraxial":
        rows = verify.gaussian_beam_vs_paraxial(fs)
        head = dict(metric="Gaussian beam: peak intensity at focus / paraxial 2 P0 / (pi w0^2) at f = 2",
                    value=rows[-1]["ratio"], unit="ratio",
                    config={"workload": "Sec. III.B.1: Gaussian envelope n = 4, Gaussian aperture tan theta0 = 1/(2f), "
                                        "R0 = 20, P0 = 1, 512^3 nodes over 40 lambda, float32, time scan R0 +- 1"})
    elif args.workload == "perturbed":
        res = verify.perturbed_focus((0.25, 0.5, 1.0, 1.5, 2.0, 3.0), runs=20)
        rows = res.pop("levels")
        head = dict(metric="flat-top pulse at f = 1: mean peak intensity / unperturbed under eps_phi = 1 "
                           "wavefront perturbations",
                    value=[r for r in rows if r["eps_phi"] == 1.0][0]["ratio_mean"], unit="ratio",
                    config={"workload": "Sec. III.B.3: Sec. III.A pulse (L = 2, eps = 0.1, R0 = 16) at f = 1, "
                                        f"{res['nbumps']} Gaussian phase bumps of width 0.3 theta, amplitudes "
                                        "uniform in +-eps_phi, 20 draws per level, D = 2 L on 96 x 512 x 512 "
                                        "nodes, float32, window following the pulse"},
                    unperturbed={k: res[k] for k in ("theta", "nbumps", "peak_intensity", "t_peak", "x_peak")},
                    samples=res["samples"])
    else:
        fs = fs + (3.0,)
        rows = verify.flattop_peak_vs_f(fs)
        head = dict(metric="flat-top pulse: peak cycle-averaged intensity at f = 0.5 (P0 = 1, lambda = 1)",
                    value=[r for r in rows if r["f_number"] == 0.5][0]["peak_intensity"], unit="P0 / lambda^2",
                    config={"workload": "Sec. III.B.2: Sec. III.A pulse (L = 2, eps = 0.1, R0 = 16), D = 2 L, "
                                        "128 x 1024 x 1024 nodes, float32, window following the pulse"})
    el = time.perf_counter() - t0
    print(json.dumps(dict(head, n_gpus=1, steps=1, warmup=0, ms_per_step=el * 1e3, higher_is_better=True,
                          scaling="weak", vs_baseline=None, dtype="f32", data="synthetic", sweep=rows)), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.workload == "c4":
        bench_c4(args)
        return
    if args.workload in ("verify", "duplicate"):
        bench_verify(args)
        return
    if args.workload in ("paraxial", "flattop", "perturbed"):
        bench_examples(args)
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

    cfg = dict(cfg, grid=grid)
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
        t_focus = focus_step * cfg["dt"]
        if not args.no_cpu_baseline:
            # outside the timed region: the oracle's start state (the init after
            # the one-time removal of longitudinal B) and the timed run's window
            import numpy as np
            s.set_pulse(cfg["pulse"])
            s.advance(1, 0.0)
            start = np.empty(s.shape, dtype=np.float32 if prec == "f32" else np.float64)
            s.get_fields(start)
            window_gpu = out.cpu().numpy()

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
    kernels = pass_kernels(tf.tf_kernel_plan(grid, prec), n[2])
    traffic = traffic_record(kernels[dom])
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
        "roofline": {"bound": "hbm", "kernel": kernels[dom], "pass": dom, "achieved": achieved, "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS,
                     "traffic": traffic, "alg_bytes_per_launch": alg_bytes},
        "focal_peak_abs": peak_field,
    }
    if not args.no_surrogate:
        line["surrogate"] = surrogate_section()
    if not args.no_cpu_baseline:
        line["cpu_baseline"], line["parity"] = cpu_baseline(start, cfg, focus_step, window_gpu, t_focus)
        del start
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
