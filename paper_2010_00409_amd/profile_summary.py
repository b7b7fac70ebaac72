"""Summaries of rocprofv3 output for the kernels of this library.

    python -m paper_2010_00409_amd.profile_summary stats DIR
        per-kernel calls, total and mean duration from a --kernel-trace run
    python -m paper_2010_00409_amd.profile_summary counters DIR [DIR ...]
        mean of every counter per dispatch, per kernel, from --pmc runs
    python -m paper_2010_00409_amd.profile_summary traffic FETCH_DIR WRITE_DIR [--json OUT]
        mean FETCH_SIZE / WRITE_SIZE (KiB per dispatch) per kernel from two
        --pmc runs, scaled by the factor that makes a plain device copy of
        known size (the largest "copy" kernel, 1 GiB read + 1 GiB write)
        read and write exactly its size
"""
import csv
import glob
import hashlib
import json
import os
import re
import sys

COPY_BYTES = 1 << 30


def _gemm_args(name):
    """Template arguments of a surrogate GEMM kernel name, demangled or not."""
    if "k_gemm<" in name:
        return name.split("k_gemm<", 1)[1].split(">(", 1)[0].replace(" ", "")
    code = name.split("k_gemmI", 1)[1].split("EEvN", 1)[0] + "E"
    words = {"f": "float", "d": "double", "DF16b": "bf16", "Lb0E": "false", "Lb1E": "true"}
    out = []
    while code and code != "E":
        m = re.match(r"Li(-?\d+)E", code)
        if m:
            out.append(m.group(1))
            code = code[m.end():]
            continue
        for k, v in words.items():
            if code.startswith(k):
                out.append(v)
                code = code[len(k):]
                break
        else:
            return name[:60]
    return ",".join(out)


def _short(name):
    if "k_gemm" in name:                      # surrogate GEMM: keep the tile shape and types
        return "k_gemm<" + _gemm_args(name) + ">"
    for key in ("k_z_fast", "k_z_wave", "k_col_fast", "k_x_forward", "k_x_inverse", "k_init_map", "k_readout",
                "k_lift_x", "k_line_fwd", "k_line_proj", "k_lineout", "k_proj", "k_head_eff",
                "k_col", "k_z", "k_sumsq", "k_reduce", "copy"):
        if key in name:
            return key
    return name[:60]


def kernel_rows(d):
    files = glob.glob(os.path.join(d, "**", "*kernel_trace.csv"), recursive=True)
    rows = []
    for f in files:
        with open(f) as fh:
            for r in csv.DictReader(fh):
                rows.append((r["Kernel_Name"], int(r["End_Timestamp"]) - int(r["Start_Timestamp"])))
    return rows


def stats(d):
    agg = {}
    for name, ns in kernel_rows(d):
        k = agg.setdefault(name, [0, 0])
        k[0] += 1
        k[1] += ns
    total = sum(v[1] for v in agg.values()) or 1
    out = ["| kernel | calls | total ms | mean us | % |", "|---|---|---|---|---|"]
    for name, (n, ns) in sorted(agg.items(), key=lambda kv: -kv[1][1]):
        out.append(f"| {_short(name)} | {n} | {ns / 1e6:.3f} | {ns / n / 1e3:.1f} | {100 * ns / total:.1f} |")
    return "\n".join(out), {n: (c, ns) for n, (c, ns) in agg.items()}


def dispatches(d, counter):
    """[(kernel name, grid size, value)] of every dispatch of a --pmc run."""
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    out = []
    for f in files:
        with open(f) as fh:
            for r in csv.DictReader(fh):
                if r.get("Counter_Name") == counter:
                    out.append((r["Kernel_Name"], int(r["Grid_Size"]), float(r["Counter_Value"])))
    return out


def counters(d, counter):
    per = {}
    for name, _, v in dispatches(d, counter):
        per.setdefault(name, []).append(v)
    return {k: sum(v) / len(v) for k, v in per.items()}


def counter_table(dirs, kernels=None):
    """Markdown table: per kernel (short name), the mean per dispatch of every
    counter found in the --pmc runs under dirs."""
    per = {}
    names = []
    for d in dirs:
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            with open(f) as fh:
                for r in csv.DictReader(fh):
                    k, c = _short(r["Kernel_Name"]), r["Counter_Name"]
                    if kernels and k not in kernels:
                        continue
                    per.setdefault(k, {}).setdefault(c, []).append(float(r["Counter_Value"]))
                    if c not in names:
                        names.append(c)
    out = ["| kernel | " + " | ".join(names) + " |", "|---|" + "---|" * len(names)]
    for k in sorted(per):
        vals = [per[k].get(c) for c in names]
        out.append(f"| {k} | " + " | ".join(f"{sum(v) / len(v):.4g}" if v else "" for v in vals) + " |")
    return "\n".join(out)


def copy_value(d, counter):
    """Mean counter value of the largest-grid copy dispatches (the 1 GiB copy)."""
    rows = [r for r in dispatches(d, counter) if "copy" in r[0].lower()]
    if not rows:
        raise SystemExit("no copy kernel in " + d)
    g = max(r[1] for r in rows)
    vals = [r[2] for r in rows if r[1] == g]
    return sum(vals) / len(vals), rows[0][0]


def kernel_sources(unit="fft_f32.hip"):
    """The files the float32 pass kernels are compiled from: the translation
    unit and the csrc headers it includes, transitively, in include order."""
    src = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
    order, todo = [], [unit]
    while todo:
        f = todo.pop(0)
        path = os.path.join(src, f)
        if f in order or not os.path.exists(path):
            continue
        order.append(f)
        todo += re.findall(r'^#include "([^"/]+)"', open(path).read(), re.M)
    return [os.path.join(src, f) for f in order]


def source_hash():
    """SHA-256 of the pass kernels' sources and their build flags (the float32
    translation units, the headers they include and build.py): counters
    recorded against it stay valid while those kernels are unchanged."""
    h = hashlib.sha256()
    paths = kernel_sources() + [p for p in kernel_sources("fft_f32_zwave.hip") if p not in kernel_sources()]
    paths.append(os.path.join(os.path.dirname(os.path.abspath(__file__)), "build.py"))
    for path in paths:
        h.update(open(path, "rb").read())
    return h.hexdigest()


def traffic(fetch_dir, write_dir):
    fe = counters(fetch_dir, "FETCH_SIZE")
    wr = counters(write_dir, "WRITE_SIZE")
    cf, ck = copy_value(fetch_dir, "FETCH_SIZE")
    cw, _ = copy_value(write_dir, "WRITE_SIZE")
    fs = (COPY_BYTES / 1024) / cf
    ws = (COPY_BYTES / 1024) / cw
    lines = [f"copy calibration: 1 GiB device copy ({_short(ck)}) reads FETCH_SIZE {cf:.0f} KiB and "
             f"WRITE_SIZE {cw:.0f} KiB per dispatch; scale factors FETCH x{fs:.4f}, WRITE x{ws:.4f}", "",
             "| kernel | FETCH KiB/dispatch | WRITE KiB/dispatch | scaled GB/dispatch (r+w) |",
             "|---|---|---|---|"]
    rec = {}
    for k in sorted(fe, key=lambda k: -fe[k]):
        f, w = fe[k], wr.get(k, 0.0)
        gb = (f * fs + w * ws) * 1024 / 1e9
        lines.append(f"| {_short(k)} | {f:.0f} | {w:.0f} | {gb:.3f} |")
        rec[_short(k)] = {"fetch_kib": f, "write_kib": w, "bytes_per_launch": (f * fs + w * ws) * 1024}
    return "\n".join(lines), rec, (fs, ws)


if __name__ == "__main__":
    mode = sys.argv[1]
    if mode == "stats":
        print(stats(sys.argv[2])[0])
    elif mode == "counters":
        print(counter_table(sys.argv[2:]))
    elif mode == "traffic":
        text, rec, _ = traffic(sys.argv[2], sys.argv[3])
        print(text)
        if "--json" in sys.argv:
            out = sys.argv[sys.argv.index("--json") + 1]
            h = source_hash()
            data = {k: dict(v, source_sha256=h) for k, v in rec.items()}
            json.dump(data, open(out, "w"), indent=1)
    else:
        raise SystemExit(__doc__)
