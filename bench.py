#!/usr/bin/env python3
"""Throughput of the Fourier-domain acceleration search on one MI355X.

One step = one fdas_search call over the whole batch: real FFT, median
normalisation, power plane, harmonic sums, thresholding, compaction, drift
argmax and the copy of the candidate list to host memory. The float32 series
are resident in HBM when the timed region starts. Prints ONE JSON line.

Default workload: the PMPS-shaped long-series batch (32 series x 2^23
samples at 250 us, zmax 200, dz 2, numharm 16, sigma 6; binary-like pulse
trains in 8 series and 50/100/150 Hz RFI tones in all), the largest
single-GPU configuration of the benchmark set (5.39e10 cells per step).
--config 2 runs the FAST drift-scan batch (128 x 2^18, numharm 8), whose
figures the default run also reports under "fast_batch".

Extra fields: "roofline" of the dominant kernel (device time per launch from
HIP events recorded by the library on the search stream; HBM roof at the
plane's 4 bytes per cell, FP32 VALU fraction beside it), "cpu_baseline" (the
FP64 oracle on a bounded sample, timed on the host cores), "plain_path" (the
same kernels driven one series at a time) and "phases_ms".
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "f-fdot cells/s (FDAS+harmsum) vs plain path at ≤1e-4 rel power error"
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP32_VECTOR_PEAK = 157.3       # TFLOP/s, 256 CUs x 2.4 GHz x 256 FP32 flop/clk
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
KERNEL_SOURCES = {"plane": "k_corr.hip", "harmsum": "k_harm.hip"}
DOMINANT = {"plane": "k_corr_power", "harmsum": "k_harm_bound"}


def _workload(config: int):
    import synth
    return {1: synth.config1, 2: synth.config2, 3: synth.config3, 4: synth.config4}[config]()


def kernel_hash(phase: str) -> str:
    src = os.path.join(ROOT, "paper_1912_12807_amd", "csrc", KERNEL_SOURCES[phase])
    h = hashlib.sha256()
    for f in (src, os.path.join(ROOT, "paper_1912_12807_amd", "csrc", "dft_small.h")):
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(phase: str, workload: str, seg_len: int = None):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if still current
    (same kernel source and, for the plane, the same segment length)."""
    try:
        with open(TRAFFIC_FILE) as fh:
            rec = json.load(fh).get(f"{workload}:{phase}")
    except (OSError, ValueError):
        return None
    if not rec or rec.get("kernel_hash") != kernel_hash(phase):
        return None
    if phase == "plane" and rec.get("seg_len") != seg_len:
        return None
    return rec.get("bytes_per_launch")


def _oracle_series(args):
    config, b = args
    import oracle as O
    import synth
    wl = _workload(config)
    x = synth.generate(wl, [b])[0]
    t0 = time.perf_counter()
    O.search_series(x, wl.tsamp, wl.zmax, wl.dz, wl.numharm, wl.sigma, series=b)
    return time.perf_counter() - t0


def _oracle_ragged_series(args):
    config, b = args
    import oracle as O
    import synth
    wl = _workload(config)
    x = synth.generate_series(wl, b)
    t0 = time.perf_counter()
    O.search_series(x, wl.tsamp[b], wl.zmax[b], wl.dz, wl.numharm, wl.sigma, series=b)
    return time.perf_counter() - t0


def _oracle_window(args):
    """Oracle time of every stage's maxima over W columns of one series of the
    long-series batch (banded direct sums), excluding the series generation."""
    config, b, W = args
    import oracle as O
    import synth
    wl = _workload(config)
    x = synth.generate(wl, [b])[0]
    t0 = time.perf_counter()
    Ah = O.normalise(O.spectrum(x))[0]
    rlo = O.rlo_bins(wl.nsamp, wl.tsamp)
    lo = 2 * rlo * wl.numharm
    ncand = 0
    for H in O.stage_list(wl.numharm):
        _, M, _ = O.band_maxima(Ah, rlo, wl.zmax, wl.dz, H, lo, lo + W)
        ncand += int((M > O.threshold(H, wl.sigma)).sum())
    return time.perf_counter() - t0, ncand


def cpu_baseline_windows(config: int, wl, nz: int, cells_total: float, W: int = 1 << 18, max_cores: int = 16):
    """The FP64 oracle on a bounded sample of the long-series batch: every stage's
    maxima of W columns of each of up to 16 series, one process per series."""
    import multiprocessing as mp
    cores = max(1, min(max_cores, len(os.sched_getaffinity(0)), wl.nseries))
    ctx = mp.get_context("spawn")
    with ctx.Pool(cores) as pool:
        res = pool.map(_oracle_window, [(config, b, W) for b in range(cores)])
    wall = max(t for t, _ in res)
    cells = cores * W * nz
    value = cells / wall
    return {"value": value, "unit": "cells/s", "cores": cores, "kind": "oracle",
            "sample": f"{cores} of {wl.nseries} series, {W} contiguous columns each (from the start of the "
                      f"stage-{wl.numharm} band) at all {nz} drift rows, every stage 1..{wl.numharm} with "
                      f"thresholds (FP64 oracle: spectrum, median normalisation and banded direct tap sums of "
                      f"the cells the harmonic sums read), one process per series; value = {cells:.3g} cells "
                      f"/ {wall:.1f} s (the slowest process, generation excluded)",
            "extrapolated_s_per_step": cells_total / value,
            "cpu": _cpu_model()}


def stream_copy_gbs(nbytes: int = 1 << 30, reps: int = 5) -> float:
    """Achievable HBM bandwidth on this GPU: a plain device-to-device copy of
    nbytes, (read + written bytes) / time, best of reps."""
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1) / 1e3)
    del a, b
    return 2.0 * nbytes / best / 1e9


def _cpu_model() -> str:
    """The host CPU as /proc/cpuinfo reports it: model name, clock, sockets and
    logical CPUs, and how many of them this process may use (on a virtual
    machine the model name can be generic)."""
    name, mhz, sockets, logical = "", "", set(), 0
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                key, _, val = line.partition(":")
                key, val = key.strip(), val.strip()
                if key == "processor":
                    logical += 1
                elif key == "model name" and not name:
                    name = val
                elif key == "cpu MHz" and not mhz:
                    mhz = val
                elif key == "physical id":
                    sockets.add(val)
    except OSError:
        return ""
    usable = len(os.sched_getaffinity(0))
    clock = f", {float(mhz) / 1e3:.2f} GHz reported" if mhz else ""
    return (f"{name}{clock}, {len(sockets) or 1} socket(s), {logical} logical CPUs, "
            f"{usable} usable by this process")


def cpu_baseline_ragged(config: int, wl, cells_of, max_cores: int = 16, max_nsamp: int = 1 << 17):
    """The FP64 oracle on the first series of at most max_nsamp samples, one process each."""
    import multiprocessing as mp
    cores = max(1, min(max_cores, len(os.sched_getaffinity(0))))
    pick = [b for b in range(wl.nseries) if wl.nsamp[b] <= max_nsamp][:cores]
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(len(pick)) as pool:
        per = pool.map(_oracle_ragged_series, [(config, b) for b in pick])
    wall = time.perf_counter() - t0
    cells = sum(cells_of[b] for b in pick)
    return {"value": cells / wall, "unit": "cells/s", "cores": len(pick), "kind": "oracle",
            "sample": f"the first {len(pick)} series of at most {max_nsamp} samples of the uneven batch "
                      f"(zmax {sorted({wl.zmax[b] for b in pick})}), one oracle process per series, "
                      f"full plane + harmonic sums + candidates in FP64 ({wall:.1f} s wall, "
                      f"{sum(per) / len(pick):.1f} s per series)",
            "cpu": _cpu_model()}


def cpu_baseline(config: int, wl, nr: int, nz: int, max_cores: int = 16):
    """The FP64 oracle, one process per series (the paper's process-level strategy)."""
    import multiprocessing as mp
    cores = max(1, min(max_cores, len(os.sched_getaffinity(0))))
    nser = min(cores, wl.nseries)
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(nser) as pool:
        per = pool.map(_oracle_series, [(config, b) for b in range(nser)])
    wall = time.perf_counter() - t0
    cells = nser * nr * nz
    model = _cpu_model()
    return {"value": cells / wall, "unit": "cells/s", "cores": nser, "kind": "oracle",
            "sample": f"{nser} of {wl.nseries} series of the same workload, one oracle process per "
                      f"series, full plane + harmonic sums + candidates in FP64 "
                      f"({wall:.1f} s wall, {sum(per) / nser:.1f} s per series)",
            "cpu": model}


# ----------------------------------------------------------------------------- profile summaries

def _kernel_key(name: str) -> str:
    return name.split("(")[0].replace("void ", "").strip()


def stats_summary(stats_csv: str, title: str, command: str) -> str:
    """Markdown table of a rocprofv3 --kernel-trace --stats CSV."""
    import csv
    rows = list(csv.DictReader(open(stats_csv)))
    out = [f"# {title}", "", "Command (repository root on the GPU host as $REPO):", "", "```", command, "```", "",
           "| kernel | calls | avg us | share % |", "|---|---|---|---|"]
    for r in rows:
        out.append(f"| `{_kernel_key(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                   f"{float(r['Percentage']):.2f} |")
    return "\n".join(out) + "\n"


def pmc_summary(fetch_csv: str, write_csv: str, workload: str, command: str):
    """HBM bytes per launch of the search kernels from FETCH_SIZE/WRITE_SIZE (KiB per dispatch).

    Each counter is scaled by what it reads for the 1 GiB device copy that
    --copy-calibration runs in the same process (known 1 GiB read, 1 GiB written).
    """
    import csv
    import collections

    def load(path):
        per = collections.defaultdict(list)
        for r in csv.DictReader(open(path)):
            per[_kernel_key(r["Kernel_Name"])].append(float(r["Counter_Value"]))
        return per

    fe, wr = load(fetch_csv), load(write_csv)
    gib_kib = float(1 << 20)
    cw = [v for v in wr.get("__amd_rocclr_copyBuffer", []) if abs(v - gib_kib) < 0.01 * gib_kib]
    cf = sorted(fe.get("__amd_rocclr_copyBuffer", []))[-len(cw):] if cw else []
    if not cw or not cf:
        raise RuntimeError("calibration copy not found in the counter output")
    f_scale = gib_kib / (sum(cf) / len(cf))
    w_scale = gib_kib / (sum(cw) / len(cw))
    res = {}
    lines = [f"# HBM traffic per launch: {workload}", "", "Commands (repository root on the GPU host as $REPO):", "",
             "```", command, "```", "",
             f"Calibration: a 1 GiB device copy reads FETCH_SIZE {sum(cf) / len(cf):.0f} KiB and WRITE_SIZE "
             f"{sum(cw) / len(cw):.0f} KiB, so FETCH is scaled by {f_scale:.3f} and WRITE by {w_scale:.3f}.", "",
             "| kernel | launches | fetched GB | written GB | total GB |", "|---|---|---|---|---|"]
    for k in sorted(set(fe) & set(wr)):
        if not k.startswith("fdas::"):
            continue
        f = sum(fe[k]) / len(fe[k]) * 1024 * f_scale
        w = sum(wr[k]) / len(wr[k]) * 1024 * w_scale
        res[k] = {"fetch_bytes": f, "write_bytes": w, "bytes_per_launch": f + w, "launches": len(fe[k])}
        lines.append(f"| `{k}` | {len(fe[k])} | {f / 1e9:.3f} | {w / 1e9:.3f} | {(f + w) / 1e9:.3f} |")
    return res, "\n".join(lines) + "\n", f_scale, w_scale


def write_traffic(res, workload, f_scale, w_scale, seg_len=None):
    """profiles/traffic.json entries for the dominant-kernel candidates, keyed by source hash."""
    try:
        with open(TRAFFIC_FILE) as fh:
            data = json.load(fh)
    except (OSError, ValueError):
        data = {}
    names = {"plane": "fdas::k_corr_power", "harmsum": "fdas::k_harm_bound"}
    for phase, prefix in names.items():
        hits = [v for k, v in res.items() if k.startswith(prefix)]
        if hits:
            data[f"{workload}:{phase}"] = {"bytes_per_launch": hits[0]["bytes_per_launch"],
                                           "fetch_bytes": hits[0]["fetch_bytes"],
                                           "write_bytes": hits[0]["write_bytes"],
                                           "fetch_scale": f_scale, "write_scale": w_scale,
                                           "kernel_hash": kernel_hash(phase),
                                           **({"seg_len": seg_len} if phase == "plane" else {})}
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)


def counters_summary(csvs, title: str, command: str, bench_log: str) -> str:
    """Markdown table of per-launch hardware counters of the plane and
    harmonic-sum kernels from rocprofv3 --pmc CSVs (one per counter pass), with
    the derived rates used in the design notes. Cells per launch come from the
    bench line of the same workload (both kernels cover one series chunk)."""
    import csv
    import collections
    cells = None
    for line in open(bench_log):
        if line.startswith("{"):
            cells = json.loads(line)["roofline"].get("cells_per_launch")
    val = collections.defaultdict(lambda: collections.defaultdict(list))
    dur = collections.defaultdict(dict)
    for path in csvs:
        for r in csv.DictReader(open(path)):
            k = _kernel_key(r["Kernel_Name"])
            if not (k.startswith("fdas::k_corr_power") or k.startswith("fdas::k_harm_bound")):
                continue
            val[k][r["Counter_Name"]].append(float(r["Counter_Value"]))
            dur[k][(path, r["Dispatch_Id"])] = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9
    out = [f"# Hardware counters per launch: {title}", "", "Commands (repository root on the GPU host as $REPO):", "",
           "```", command, "```", "",
           "Averages per launch over the dispatches of every pass. GRBM_GUI_ACTIVE is summed over the 8 XCDs and "
           "SQ_BUSY_CYCLES over the 32 shader engines; 'GRBM clock' = GRBM_GUI_ACTIVE / 8 / launch time. VALU "
           "per cell = SQ_INSTS_VALU x 64 lanes / plane cells of the launch "
           f"({cells:.4g} cells per launch). L2 hit rate = TCC_HIT / (TCC_HIT + TCC_MISS). Busy fractions "
           "are per unit over the GRBM cycles of the launch (1024 SIMDs, 256 scalar units and 256 texture "
           "addressers); the counters come from separate passes, so rates that mix passes assume the "
           "passes ran alike (their launch times agree within a few per cent).", ""]
    for k in sorted(val):
        c = {n: sum(v) / len(v) for n, v in val[k].items()}
        t = sum(dur[k].values()) / len(dur[k])
        out += [f"## `{k}`", "", f"launch time under the counters: {t * 1e3:.3f} ms", "",
                "| counter | per launch |", "|---|---|"]
        out += [f"| {n} | {c[n]:.4g} |" for n in sorted(c)]
        der = []
        g = c.get("GRBM_GUI_ACTIVE")
        if g:
            der.append(("GRBM clock (GHz)", g / 8 / t / 1e9))
        if "SQ_INSTS_VALU" in c:
            if cells:
                der.append(("VALU instructions per cell (lanes)", c["SQ_INSTS_VALU"] * 64 / cells))
            if c.get("SQ_WAVES"):
                der.append(("VALU instructions per wave", c["SQ_INSTS_VALU"] / c["SQ_WAVES"]))
            if g:
                der.append(("VALU instructions per SIMD per GRBM cycle", c["SQ_INSTS_VALU"] / (1024 * g / 8)))
            if g:
                der.append(("VALU busy fraction (4 cycles per wave64 instruction)",
                            4 * c["SQ_INSTS_VALU"] / (1024 * g / 8)))
        if "SQ_INSTS_SALU" in c and g:
            der.append(("SALU busy fraction (one scalar unit per CU)", c["SQ_INSTS_SALU"] / (256 * g / 8)))
        if "TA_BUSY_avr" in c and g:
            der.append(("texture addresser busy fraction", c["TA_BUSY_avr"] / (g / 8)))
            if "SQ_INSTS_VMEM_RD" in c:
                der.append(("texture addresser cycles per vector memory read",
                            c["TA_BUSY_avr"] / (c["SQ_INSTS_VMEM_RD"] / 256)))
        if "SQ_BUSY_CYCLES" in c and g:
            der.append(("SQ busy fraction", c["SQ_BUSY_CYCLES"] / (4 * g)))
        if "SQ_ACTIVE_INST_VALU" in c and g:
            der.append(("VALU active cycles per SIMD / GRBM cycles", c["SQ_ACTIVE_INST_VALU"] / (1024 * g / 8)))
        if "SQ_INSTS_VMEM_RD" in c and c.get("SQ_WAVES"):
            der.append(("vector memory reads per wave", c["SQ_INSTS_VMEM_RD"] / c["SQ_WAVES"]))
        if "TCC_HIT_sum" in c and "TCC_MISS_sum" in c:
            der.append(("L2 hit rate", c["TCC_HIT_sum"] / max(1.0, c["TCC_HIT_sum"] + c["TCC_MISS_sum"])))
        if "TCP_TCC_READ_REQ_LATENCY_sum" in c and c.get("TCP_TCC_READ_REQ_sum"):
            der.append(("mean L1-to-L2 read latency (cycles)",
                        c["TCP_TCC_READ_REQ_LATENCY_sum"] / c["TCP_TCC_READ_REQ_sum"]))
        if der:
            out += ["", "| derived | value |", "|---|---|"] + [f"| {n} | {v:.4g} |" for n, v in der]
        out.append("")
    return "\n".join(out)


def launch_tails_summary(trace_csv: str, title: str, command: str, steps: int) -> str:
    """Markdown summary of what grouped launches cost beyond their work, from a
    rocprofv3 --kernel-trace CSV of eager searches.

    Per kernel family, the launch with the most workgroups sets the time per
    workgroup; every launch's excess over (its workgroups x that time) is its
    tail (an under-filled machine at the start and end of a small launch). Gaps
    are idle device time between consecutive kernels of the timed searches."""
    import csv
    rows = [r for r in csv.DictReader(open(trace_csv)) if r.get("Kind", "KERNEL_DISPATCH") == "KERNEL_DISPATCH"]
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    fam = {}
    for r in rows:
        name = _kernel_key(r["Kernel_Name"])
        if not name.startswith("fdas::"):
            continue
        wg = (int(r["Grid_Size_X"]) // max(1, int(r["Workgroup_Size_X"]))) * int(r["Grid_Size_Y"]) * \
            int(r["Grid_Size_Z"])
        dur = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-6   # ms
        fam.setdefault(name, []).append((wg, dur, int(r["Start_Timestamp"]), int(r["End_Timestamp"])))
    out = [f"# Launch tails: {title}", "", "Command (repository root on the GPU host as $REPO):", "", "```", command,
           "```", "",
           "Per kernel family, the largest launch's time per workgroup is taken as the full-machine rate; a "
           "launch's tail is its duration minus its workgroups at that rate. Gaps: idle device time between "
           "consecutive kernels. Figures per search.", "",
           "| kernel | launches per search | ms per search | tail ms per search | tail % of kernel |",
           "|---|---|---|---|---|"]
    total_ms = total_tail = 0.0
    for name, ls in sorted(fam.items(), key=lambda kv: -sum(d for _, d, _, _ in kv[1])):
        big = max(ls, key=lambda x: x[0])
        rate = big[1] / max(1, big[0])
        dur = sum(d for _, d, _, _ in ls)
        tail = sum(max(0.0, d - w * rate) for w, d, _, _ in ls)
        total_ms += dur
        total_tail += tail
        out.append(f"| `{name}` | {len(ls) / steps:.1f} | {dur / steps:.3f} | {tail / steps:.3f} | "
                   f"{100 * tail / max(dur, 1e-12):.1f} |")
    spans = sorted((a, b) for ls in fam.values() for _, _, a, b in ls)
    busy = gaps = 0.0
    cur_a, cur_b = spans[0]
    for a_, b_ in spans[1:]:
        if a_ > cur_b:
            busy += (cur_b - cur_a) * 1e-6
            gaps += (a_ - cur_b) * 1e-6
            cur_a, cur_b = a_, b_
        else:
            cur_b = max(cur_b, b_)
    busy += (cur_b - cur_a) * 1e-6
    out += ["", f"Kernels {total_ms / steps:.3f} ms per search, of which tails {total_tail / steps:.3f} ms "
                f"({100 * total_tail / total_ms:.1f} %); device busy {busy / steps:.3f} ms, gaps between kernels "
                f"{gaps / steps:.3f} ms per search (gaps include the host work between searches)."]
    return "\n".join(out) + "\n"


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=3, choices=(1, 2, 3, 4, 5, 6, 7))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the FAST-batch figures of the default run")
    ap.add_argument("--eager-only", action="store_true",
                    help="config 4: only warmup + steps eager grouped searches (for kernel traces)")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--autotune", type=int, default=0, choices=(0, 1),
                    help="time candidate launch parameters on the first search (during warmup)")
    ap.add_argument("--seg-len", type=int, default=0, help="plan option seg_len (0: the plan's choice)")
    ap.add_argument("--harm-block", type=int, default=0, help="plan option harm_block (0: default)")
    ap.add_argument("--harm-pair", type=int, default=0, choices=(0, 1, 2),
                    help="plan option harm_pair (0 automatic, 1 maxima per column, 2 per bin)")
    ap.add_argument("--tuning", default="",
                    help="launch parameters to preload, tuning lines separated by ';' (no tuning for those shapes)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (scale for HBM byte counters)")
    ap.add_argument("--stats-summary", nargs=3, metavar=("STATS_CSV", "OUT_MD", "COMMAND"),
                    help="write a markdown summary of a rocprofv3 kernel-stats CSV and exit")
    ap.add_argument("--summary-title", default="",
                    help="workload description for --stats-summary (default: the config's workload name)")
    ap.add_argument("--counters-summary", nargs="+", metavar="ARG",
                    help="OUT_MD COMMAND BENCH_LOG CSV [CSV ...]: per-launch counters of the plane and "
                         "harmonic-sum kernels (title from --summary-title)")
    ap.add_argument("--tails-summary", nargs=4, metavar=("TRACE_CSV", "OUT_MD", "COMMAND", "SEARCHES"),
                    help="write the launch-tail summary of a rocprofv3 kernel trace and exit")
    ap.add_argument("--pmc-summary", nargs=4, metavar=("FETCH_CSV", "WRITE_CSV", "OUT_MD", "COMMAND"),
                    help="summarise FETCH_SIZE/WRITE_SIZE runs into OUT_MD and profiles/traffic.json")
    ap.add_argument("--pmc-seg-len", type=int, default=2048,
                    help="segment length the counter runs used (recorded with the plane traffic)")
    args = ap.parse_args()
    if args.stats_summary:
        csv_path, out_md, cmd = args.stats_summary
        title = args.summary_title or _workload(args.config).name
        with open(out_md, "w") as fh:
            fh.write(stats_summary(csv_path, f"Kernel time summary: {title}", cmd))
        return
    if args.tails_summary:
        csv_path, out_md, cmd, n = args.tails_summary
        title = args.summary_title or _workload(args.config).name
        with open(out_md, "w") as fh:
            fh.write(launch_tails_summary(csv_path, title, cmd, int(n)))
        return
    if args.counters_summary:
        if len(args.counters_summary) < 4:
            ap.error("--counters-summary needs OUT_MD COMMAND BENCH_LOG CSV [CSV ...]")
        out_md, cmd, log = args.counters_summary[:3]
        title = args.summary_title or _workload(args.config).name
        with open(out_md, "w") as fh:
            fh.write(counters_summary(args.counters_summary[3:], title, cmd, log))
        return
    if args.pmc_summary:
        fcsv, wcsv, out_md, cmd = args.pmc_summary
        wl = _workload(args.config)
        res, md, fs, ws = pmc_summary(fcsv, wcsv, wl.name, cmd)
        with open(out_md, "w") as fh:
            fh.write(md)
        write_traffic(res, wl.name, fs, ws, args.pmc_seg_len)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: the search is measured on one GPU only; series shard across "
              "GPUs without communication (see the design notes), but no multi-GPU figure is "
              "produced here", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1912_12807_amd as fdas
    import synth

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    fdas.load()
    if args.config == 4:
        return bench_ragged(args)
    if args.config == 5:
        return bench_refine(args)
    if args.config in (6, 7):
        return bench_pipeline(args)
    wl = _workload(args.config)
    popts = dict(seg_len=args.seg_len, harm_block=args.harm_block, harm_pair=args.harm_pair)
    res = bench_batch(wl, args, popts, copy_calibration=args.copy_calibration)
    x, cells, nr, nz = res.pop("_x"), res["cells"], res.pop("_nr"), res.pop("_nz")

    plain = None
    if not args.no_plain:
        print("[bench] plain per-series path", file=sys.stderr, flush=True)
        p1 = fdas.Plan(wl.nsamp, 1, wl.zmax, wl.dz, wl.numharm)
        p1.search(x[0:1], wl.tsamp, sigma=wl.sigma, cap=1 << 22, allow_trunc=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for b in range(wl.nseries):
            p1.search(x[b:b + 1], wl.tsamp, sigma=wl.sigma, cap=1 << 22, allow_trunc=True)
        torch.cuda.synchronize()
        pw = time.perf_counter() - t0
        plain = {"value": cells / pw, "unit": "cells/s", "ms_per_step": 1e3 * pw,
                 "what": "same kernels, one series per fdas_search call"}
        p1.close()
    del x
    torch.cuda.empty_cache()

    extra = None
    if args.config == 3 and not args.no_extra:
        # the FAST drift-scan batch with the same code, reported beside the headline
        wl2 = _workload(2)
        r2 = bench_batch(wl2, args, {}, copy_calibration=False)
        del r2["_x"], r2["_nr"], r2["_nz"]
        extra = {"workload": wl2.name, "value": r2["value"], "unit": "cells/s", "ms_per_step": r2["ms_per_step"],
                 "cells_per_step": r2["cells"], "roofline": r2["roofline"], "phases_ms": r2["phases_ms"],
                 "candidates": r2["candidates"]}
        torch.cuda.empty_cache()

    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        if args.config == 3:
            cpu = cpu_baseline_windows(args.config, wl, nz, cells)
        else:
            cpu = cpu_baseline(args.config, wl, nr, nz)

    out = {
        "metric": METRIC, "value": res["value"], "unit": "cells/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": res["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": wl.name, "nseries": wl.nseries, "nsamp": wl.nsamp, "tsamp": wl.tsamp,
                   "zmax": wl.zmax, "dz": wl.dz, "numharm": wl.numharm, "sigma": wl.sigma,
                   "cells_per_step": cells, "seg_len": res["seg_len"], "tuning": res["tuning"],
                   "parallelism": "single GPU"},
        "roofline": res["roofline"],
        "cpu_baseline": cpu,
        "plain_path": plain,
        "speedup_vs_plain": (res["value"] / plain["value"]) if plain else None,
        "phases_ms": res["phases_ms"],
        "candidates": res["candidates"],
        "fast_batch": extra,
    }
    print(json.dumps(out), flush=True)


def bench_batch(wl, args, popts, copy_calibration=False):
    """Time args.steps searches of a fixed-length batch, then the per-phase kernel
    times on a profiled plan with the same launch parameters; the roofline of the
    dominant kernel."""
    import numpy as np
    import torch

    import paper_1912_12807_amd as fdas
    import synth

    print(f"[bench] generating {wl.name}", file=sys.stderr, flush=True)
    x = torch.from_numpy(synth.generate_parallel(wl)).cuda()
    rlo, nr, nz = fdas.geometry(wl.nsamp, wl.tsamp, wl.zmax, wl.dz)
    cells = wl.nseries * nr * nz
    plan = fdas.Plan(wl.nsamp, wl.nseries, wl.zmax, wl.dz, wl.numharm, autotune=args.autotune, **popts)
    if args.tuning:
        plan.load_tuning(args.tuning.replace(";", "\n"))
    if copy_calibration:
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    print(f"[bench] {wl.name}: warmup {args.warmup}", file=sys.stderr, flush=True)
    # the long-series batch lists millions of candidates (RFI tones and their
    # harmonics): the copy-out keeps the first cap, every count is exact
    cap = 1 << 22
    for _ in range(args.warmup):
        cands, ncand = plan.search(x, wl.tsamp, sigma=wl.sigma, cap=cap, allow_trunc=True)
    torch.cuda.synchronize()
    print(f"[bench] {wl.name}: timing {args.steps} steps", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        cands, ncand = plan.search(x, wl.tsamp, sigma=wl.sigma, cap=cap, allow_trunc=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    tuning = plan.tuning().strip()
    info = plan.info()
    plan.close()
    ms_step = 1e3 * wall / args.steps
    value = cells * args.steps / wall

    # per-phase kernel times (HIP events on the search stream) from a plan with
    # the same launch parameters and profiling on, which runs every phase in
    # order on the one stream
    print(f"[bench] {wl.name}: phase timing {args.steps} steps", file=sys.stderr, flush=True)
    pplan = fdas.Plan(wl.nsamp, wl.nseries, wl.zmax, wl.dz, wl.numharm, profile=1, **popts)
    if tuning:
        pplan.load_tuning(tuning)
    pc, _ = pplan.search(x, wl.tsamp, sigma=wl.sigma, cap=cap, allow_trunc=True)
    torch.cuda.synchronize()
    pplan.profile(reset=True)
    for _ in range(args.steps):
        pplan.search(x, wl.tsamp, sigma=wl.sigma, cap=cap, allow_trunc=True)
    torch.cuda.synchronize()
    prof = pplan.profile(reset=True)
    pplan.close()
    assert np.array_equal(pc, cands), "the profiled plan found other candidates"

    phases = {k: v[0] / args.steps for k, v in prof.items()}
    dom = max(("plane", "harmsum"), key=lambda k: prof[k][0])
    roof = roofline(wl, dom, prof, args.steps, info, rlo, nr, nz, cells)
    return {"_x": x, "_nr": nr, "_nz": nz, "cells": cells, "value": value, "ms_per_step": ms_step,
            "seg_len": info["seg_len"], "tuning": tuning or None, "roofline": roof,
            "phases_ms": {k: round(v, 4) for k, v in phases.items()}, "candidates": int(ncand)}


def roofline(wl, dom, prof, steps, info, rlo, nr, nz, cells):
    """Roofline of the dominant kernel from its per-launch device time.

    Plane (K4): the path's binding roof is HBM; the kernel's algorithmic bytes are
    the 4-byte power of every cell it writes (the spectrum it reads is < 0.1 B per
    cell). Its FP32 work per cell (inverse FFTs, template products and powers,
    forward FFTs) is reported beside it against the vector peak.
    Harmonic sums (K5): the half-precision block maxima read once and the stage
    maxima written."""
    launches = max(1, prof[dom][1])
    t_launch = prof[dom][0] / 1e3 / launches           # s
    per_launch = launches / steps                      # launches of the kernel per search
    cells_launch = cells / per_launch
    L, mseg = info["seg_len"], info["mseg"]
    NS = int(math.log2(wl.numharm)) + 1
    if dom == "plane":
        byts = 4.0 * cells_launch
        flops = plane_flops(wl.nseries / per_launch, wl.nsamp, rlo, nz, L, mseg)
        alu = flops / t_launch / 1e12
        achieved = byts / t_launch / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "kernel": DOMINANT[dom], "per_unit": "4 B/cell (plane write)",
                "cells_per_launch": cells_launch,
                "alu": {"achieved": alu, "peak": FP32_VECTOR_PEAK, "unit": "TFLOP/s",
                        "frac": alu / FP32_VECTOR_PEAK, "per_unit": f"{flops / cells_launch:.1f} FLOP/cell",
                        "nonpacked_peak": FP32_VECTOR_PEAK / 2,
                        "frac_of_nonpacked": alu / (FP32_VECTOR_PEAK / 2)}}
    else:
        ser = wl.nseries / per_launch
        mp_ = (nr + 15) // 16 * 16
        if info["harm_blocks"]:
            # bounded sums read the drift-block maxima (2-byte halves) once and
            # write the stage maxima (4-byte floats)
            ncols = nr // 2 if info["harm_pair"] else nr
            byts = ser * (info["harm_blocks"] * ncols * 2.0 + NS * mp_ * 4.0)
        else:
            byts = cells_launch * 4.0 + ser * NS * mp_ * 4.0
        achieved = byts / t_launch / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "kernel": DOMINANT[dom] if info["harm_blocks"] else "k_harmsum",
                "per_unit": f"{byts / cells_launch:.3f} B/cell", "cells_per_launch": cells_launch}
    roof["traffic"] = measured_traffic(dom, wl.name, L)
    roof["launch_ms"] = t_launch * 1e3
    roof["stream_copy_gbs"] = stream_copy_gbs()
    return roof


def plane_flops(nseries, nsamp, rlo, nz, L, mseg):
    # nseries may be fractional: the series share of one launch
    """Algorithmic FLOPs of the overlap-save plane: per (z row, parity, segment) an inverse
    FFT (5 L log2 L), the template product (6 L) and the power (3 L); per segment and z
    group one forward FFT and the scaling."""
    Lv = L - 2 * mseg
    nseg = math.ceil((nsamp // 2 - rlo) / Lv)
    G = 1
    while G < 8 and nz >= 2 * G * 12:
        G *= 2
    return nseries * nseg * (2 * nz * (5 * L * math.log2(L) + 9 * L) + G * (5 * L * math.log2(L) + 2 * L))


def bench_ragged(args):
    """Uneven batch: 512 series of 2^16..2^20 samples with per-series zmax in one
    fdas_search_ragged call (graph replay, autotuned launch parameters), against
    the plain path (one fdas_search call per series, default parameters)."""
    import numpy as np
    import torch

    import paper_1912_12807_amd as fdas
    import synth

    wl = _workload(4)
    print(f"[bench] generating {wl.name}", file=sys.stderr, flush=True)
    offs = wl.offsets()
    buf = torch.from_numpy(synth.generate_ragged(wl)).cuda()
    geo = [fdas.geometry(wl.nsamp[b], wl.tsamp[b], wl.zmax[b], wl.dz) for b in range(wl.nseries)]
    cells_of = [nr * nz for _, nr, nz in geo]
    cells = float(sum(cells_of))
    nmax, zmax = max(wl.nsamp), max(wl.zmax)
    run = dict(sigma=wl.sigma, cap=1 << 21)

    def call(plan):
        return plan.search_ragged(buf, offs, wl.nsamp, wl.tsamp, wl.zmax, **run)

    def timed(plan, steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            c = call(plan)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps, c

    if args.eager_only:
        # only warmup + steps eager grouped searches with the given launch parameters
        # (for kernel traces: nothing else runs on the device)
        plan = fdas.Plan(nmax, wl.nseries, zmax, wl.dz, wl.numharm)
        if args.tuning:
            plan.load_tuning(args.tuning.replace(";", "\n"))
        for _ in range(args.warmup):
            call(plan)
        sec, cands = timed(plan, args.steps)
        print(json.dumps({"workload": wl.name, "eager_ms_per_search": 1e3 * sec, "searches": args.warmup + args.steps,
                          "cells_per_step": cells, "candidates": int(len(cands))}), flush=True)
        return

    plan = fdas.Plan(nmax, wl.nseries, zmax, wl.dz, wl.numharm, autotune=1, graph=1)
    if args.tuning:
        plan.load_tuning(args.tuning.replace(";", "\n"))
    print(f"[bench] warmup {args.warmup} (autotune, graph capture)", file=sys.stderr, flush=True)
    for _ in range(max(1, args.warmup)):
        cands = call(plan)
    tuning = plan.tuning()
    print(f"[bench] timing {args.steps} steps", file=sys.stderr, flush=True)
    sec, cands = timed(plan, args.steps)
    value = cells / sec

    # same launches eagerly with phase events: kernel times for the roofline
    prof = fdas.Plan(nmax, wl.nseries, zmax, wl.dz, wl.numharm, profile=1)
    prof.load_tuning(tuning)
    call(prof)
    prof.profile(reset=True)
    pe_sec, cands_eager = timed(prof, 2)
    ph = prof.profile(reset=True)
    assert np.array_equal(cands, cands_eager), "graph replay and eager launches disagree"
    prof.close()
    cfg = {}
    for line in tuning.split("\n"):
        f = line.split()
        if f:
            cfg[(int(f[0]), int(f[1]))] = (int(f[3]), int(f[4]), int(f[5]))
    flops = 0.0
    for b in range(wl.nseries):
        rlo, nr, nz = geo[b]
        L = cfg[(wl.nsamp[b], nz // 2)][0]
        mseg = int(math.ceil(wl.zmax[b] / 2 - 1e-9)) + 16
        flops += plane_flops(1, wl.nsamp[b], rlo, nz, L, mseg)
    k4_s = ph["plane"][0] / 1e3 / 2
    achieved = flops / k4_s / 1e12
    roof = {"bound": "alu", "achieved": achieved, "peak": FP32_VECTOR_PEAK, "unit": "TFLOP/s",
            "frac": achieved / FP32_VECTOR_PEAK, "kernel": DOMINANT["plane"],
            "per_unit": f"{flops / cells:.1f} FLOP/cell (summed over the launches of all groups)",
            "traffic": measured_traffic("plane", wl.name), "launch_ms": 1e3 * k4_s / (ph["plane"][1] / 2),
            "launches_per_step": ph["plane"][1] // 2}

    # grouped launches with default parameters, no graph
    base = fdas.Plan(nmax, wl.nseries, zmax, wl.dz, wl.numharm)
    call(base)
    b_sec, _ = timed(base, max(1, args.steps // 2))
    base.close()

    plain = None
    if not args.no_plain:
        print("[bench] plain per-series path", file=sys.stderr, flush=True)
        p1 = fdas.Plan(nmax, 1, zmax, wl.dz, wl.numharm)
        views = [buf[offs[b]:offs[b] + wl.nsamp[b]].view(1, -1) for b in range(wl.nseries)]
        p1.search(views[0], wl.tsamp[0], zmax=wl.zmax[0], **run)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for b in range(wl.nseries):
            p1.search(views[b], wl.tsamp[b], zmax=wl.zmax[b], **run)
        torch.cuda.synchronize()
        pw = time.perf_counter() - t0
        plain = {"value": cells / pw, "unit": "cells/s", "ms_per_step": 1e3 * pw,
                 "what": "same kernels, one fdas_search call per series, default launch parameters"}
        p1.close()

    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        cpu = cpu_baseline_ragged(4, wl, cells_of)

    out = {
        "metric": METRIC, "value": value, "unit": "cells/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * sec, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": wl.name, "nseries": wl.nseries, "nsamp": "2^16..2^20 (per series)",
                   "tobs_s": 52.4288, "zmax": "0/50/100/200/300 (per series)", "dz": wl.dz,
                   "numharm": wl.numharm, "sigma": wl.sigma, "cells_per_step": cells,
                   "groups": len(cfg), "parallelism": "single GPU"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "plain_path": plain,
        "speedup_vs_plain": (value / plain["value"]) if plain else None,
        "grouped_default_eager": {"value": cells / b_sec, "ms_per_step": 1e3 * b_sec},
        "phases_ms": {k: round(v[0] / 2, 4) for k, v in ph.items()},
        "tuning": tuning.strip().split("\n"),
        "candidates": int(len(cands)),
    }
    print(json.dumps(out), flush=True)


def _oracle_refine(args):
    import oracle as O
    import synth
    starts, dz = args
    wl = synth.config1()
    Ah = O.normalise(O.spectrum(synth.generate(wl)[0]))[0]
    t0 = time.perf_counter()
    for r0, z0 in starts:
        O.refine(Ah, r0, z0, dz)
    return time.perf_counter() - t0


def refine_starts_gpu(plane, rlo, Z, count):
    """The count largest local maxima of a stage-1 plane on its integer-r cells (3x3 on
    that sub-grid), as (R, Zq) in decreasing power (input preparation with torch ops)."""
    import torch
    sub = plane[0][:, 0::2].contiguous()
    pad = torch.nn.functional.pad(sub[None, None], (1, 1, 1, 1), value=float("-inf"))
    mx = torch.nn.functional.max_pool2d(pad, 3, stride=1)[0, 0]
    vals = torch.where(sub >= mx, sub, torch.full_like(sub, float("-inf"))).flatten()
    top = torch.topk(vals, count)
    zi = (top.indices // sub.shape[1]).cpu().numpy()
    ji = (top.indices % sub.shape[1]).cpu().numpy()
    return [(int(2 * rlo + 2 * j), int(z - Z)) for z, j in zip(zi, ji)]


def bench_refine(args):
    """4096 starts (the largest integer-r local maxima of the single-series plane)
    refined by 20 ascent steps each, in one fdas_refine call."""
    import numpy as np
    import torch

    import paper_1912_12807_amd as fdas
    import synth

    wl = synth.config1()
    x = torch.from_numpy(synth.generate(wl)).cuda()
    rlo, nr, nz = fdas.geometry(wl.nsamp, wl.tsamp, wl.zmax, wl.dz)
    plan = fdas.Plan(wl.nsamp, 1, wl.zmax, wl.dz, 1, profile=1)
    starts = refine_starts_gpu(plan.plane(x, wl.tsamp), rlo, nz // 2, 4096)
    r0 = np.array([s[0] / 2 for s in starts])
    z0 = np.array([s[1] * wl.dz for s in starts])
    iters = 20
    print(f"[bench] refine warmup {args.warmup}", file=sys.stderr, flush=True)
    for _ in range(max(1, args.warmup)):
        r, z, P = plan.refine(x, r0, z0, iters=iters)
    plan.profile(reset=True)
    print(f"[bench] timing {args.steps} steps", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r, z, P = plan.refine(x, r0, z0, iters=iters)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / args.steps
    ph = plan.profile(reset=True)
    k_s = ph["refine"][0] / 1e3 / args.steps
    # algorithmic work: per evaluation, nodes x (8 FLOP per tap of the Horner sums + per
    # 16-tap block and node one phase reduction and sincos, counted as 20 FLOP)
    flops = 0.0
    for z_ in z0:
        M = int(math.ceil((abs(z_) + 2 * wl.dz) / 2)) + 16 + 1
        taps16 = (2 * M + 1 + 15) // 16 * 16
        npan_est = M + 1 + abs(z_) / 2 + 1
        flops += (iters + 1) * 16 * math.ceil(npan_est) * (8 * taps16 + 20 * taps16 / 16 + 30)
    achieved = flops / k_s / 1e12
    inj = wl.injections[0]
    near = np.nonzero((np.abs(r0 - inj.r0) <= 1) & (np.abs(z0 - inj.z0) <= 2 * wl.dz))[0]
    found = None
    if near.size:
        i = int(near[0])
        found = {"r": float(r[i]), "z": float(z[i]), "power": float(P[i]), "r0": inj.r0, "z0": inj.z0}
    cpu = None
    if not args.no_cpu_baseline:
        import multiprocessing as mp
        cores = max(1, min(16, len(os.sched_getaffinity(0))))
        per = 8
        sample = [list(zip(r0[i * per:(i + 1) * per], z0[i * per:(i + 1) * per])) for i in range(cores)]
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        t1 = time.perf_counter()
        with mp.get_context("spawn").Pool(cores) as pool:
            times = pool.map(_oracle_refine, [(s_, wl.dz) for s_ in sample])
        wall = time.perf_counter() - t1
        cpu = {"value": cores * per / wall, "unit": "candidates/s", "cores": cores, "kind": "oracle",
               "sample": f"the first {cores * per} of the 4096 starts, {per} per process, FP64 oracle "
                         f"ascent of 20 steps ({wall:.1f} s wall incl. start-up, "
                         f"{sum(times) / cores:.1f} s of refinement per process)",
               "cpu": _cpu_model()}
    out = {
        "metric": "refined candidates/s (20 ascent steps at fractional r, z)", "value": len(starts) / sec,
        "unit": "candidates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * sec, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 (phases and node sums f64)", "data": "synthetic",
        "config": {"workload": "refine-4096-starts-of-1x2^17", "starts": len(starts), "iters": iters,
                   "nsamp": wl.nsamp, "zmax": wl.zmax, "dz": wl.dz, "parallelism": "single GPU"},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP32_VECTOR_PEAK, "unit": "TFLOP/s",
                     "frac": achieved / FP32_VECTOR_PEAK, "kernel": "k_refine_ascent",
                     "per_unit": f"{flops / len(starts):.3g} FLOP/candidate", "traffic": None,
                     "launch_ms": 1e3 * k_s},
        "cpu_baseline": cpu,
        "injected_signal": found,
        "phases_ms": {k: round(v[0] / args.steps, 4) for k, v in ph.items()},
    }
    print(json.dumps(out), flush=True)


def _oracle_dedisp(args):
    import oracle as O
    import synth
    config, r, dm_lo, count = args
    fb = synth.fast_filterbank() if config == 6 else synth.pmps_filterbank()
    x = synth.generate_filterbank(fb)
    a, s, n, d = fb.plan[r]
    t0 = time.perf_counter()
    O.dedisperse(x, fb.freqs(), fb.tsamp, [a + (dm_lo + i) * s for i in range(count)], d)
    return time.perf_counter() - t0


def bench_pipeline(args):
    """Filterbank -> dedispersion over the paper's DM plan -> one ragged search of all trials.
    Config 6: FAST file shape with Table 3; config 7: PMPS file shape with Table 2."""
    import numpy as np
    import torch

    import paper_1912_12807_amd as fdas
    import synth

    fb = synth.fast_filterbank() if args.config == 6 else synth.pmps_filterbank()
    print(f"[bench] generating {fb.name}", file=sys.stderr, flush=True)
    fil = torch.from_numpy(synth.generate_filterbank(fb)).cuda()
    ndm = sum(n for _, _, n, _ in fb.plan)
    n_max = fb.nsamp // min(d for _, _, _, d in fb.plan)
    zmax, numharm = 50.0, 8
    plan = fdas.Plan(n_max, ndm, zmax, 2.0, numharm, autotune=1, graph=1, profile=0)
    if args.tuning:
        plan.load_tuning(args.tuning.replace(";", "\n"))
    dd = fdas.Plan(1 << 12, 1, 0.0, 2.0, 1, profile=1)
    trial_samples = sum(n * (fb.nsamp // d) for _, _, n, d in fb.plan)
    adds = sum(n * fb.nchan * (fb.nsamp // d) for _, _, n, d in fb.plan)
    print(f"[bench] warmup {args.warmup}", file=sys.stderr, flush=True)
    for _ in range(max(1, args.warmup)):
        buf, series = dd.dedisperse(fil, fb.tsamp, fb.f0, fb.df, fb.plan)
    dd.profile(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        buf, series = dd.dedisperse(fil, fb.tsamp, fb.f0, fb.df, fb.plan)
    torch.cuda.synchronize()
    dd_sec = (time.perf_counter() - t0) / args.steps
    ph = dd.profile(reset=True)
    k_dd = ph["dedisperse"][0] / 1e3 / args.steps
    offs, ns, ts = [], [], []
    o = 0
    for (a, s_, n, d), sr in zip(fb.plan, series):
        for i in range(n):
            offs.append(o + i * sr.shape[1])
            ns.append(sr.shape[1])
            ts.append(fb.tsamp * d)
        o += n * sr.shape[1]
    run = dict(dz=2.0, numharm=numharm, sigma=6.0, cap=1 << 22, allow_trunc=True)
    cells = sum(fdas.geometry(n_, t_, zmax, 2.0)[1] * fdas.geometry(n_, t_, zmax, 2.0)[2] for n_, t_ in zip(ns, ts))
    for _ in range(max(1, args.warmup)):
        cands, ncand = plan.search_ragged(buf, offs, ns, ts, zmax, **run)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        cands, ncand = plan.search_ragged(buf, offs, ns, ts, zmax, **run)
    torch.cuda.synchronize()
    s_sec = (time.perf_counter() - t0) / args.steps
    # end to end: both stages back to back
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        buf2, _ = dd.dedisperse(fil, fb.tsamp, fb.f0, fb.df, fb.plan)
        cands, ncand = plan.search_ragged(buf2, offs, ns, ts, zmax, **run)
    torch.cuda.synchronize()
    e_sec = (time.perf_counter() - t0) / args.steps
    cpu = None
    if not args.no_cpu_baseline:
        import multiprocessing as mp
        cores = max(1, min(16, len(os.sched_getaffinity(0))))
        r_big = max(range(len(fb.plan)), key=lambda r: fb.plan[r][2] * fb.nsamp // fb.plan[r][3])
        a, s_, n, d = fb.plan[r_big]
        per = max(1, min(n // cores, 8))
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        t1 = time.perf_counter()
        with mp.get_context("spawn").Pool(cores) as pool:
            times = pool.map(_oracle_dedisp, [(args.config, r_big, k * per, per) for k in range(cores)])
        wall = max(times)
        done = cores * per * (fb.nsamp // d)
        cpu = {"value": done / wall, "unit": "trial-samples/s", "cores": cores, "kind": "oracle",
               "sample": f"{cores * per} trial DMs of plan range {r_big + 1} (downsampling {d}), {per} per "
                         f"process, exact integer oracle; dedispersion time only ({wall:.2f} s, the slowest "
                         f"process)", "cpu": _cpu_model()}
    out = {
        "metric": "dedispersed trial-samples/s (filterbank to DM-trial series)", "value": trial_samples / dd_sec,
        "unit": "trial-samples/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * dd_sec, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u8 in, f32 (exact integers) out", "data": "synthetic",
        "config": {"workload": fb.name + "-dedisp", "nchan": fb.nchan, "nsamp": fb.nsamp, "tsamp": fb.tsamp,
                   "band_mhz": [float(min(fb.freqs())), float(max(fb.freqs()))], "trial_dms": ndm,
                   "plan": fb.plan, "parallelism": "single GPU"},
        "roofline": {"bound": "alu", "achieved": adds / k_dd / 1e12, "peak": FP32_VECTOR_PEAK, "unit": "TFLOP/s",
                     "frac": adds / k_dd / 1e12 / FP32_VECTOR_PEAK, "kernel": "k_dedisperse",
                     "per_unit": f"{fb.nchan} adds per trial-sample", "traffic": None,
                     "launch_ms": 1e3 * k_dd},
        "cpu_baseline": cpu,
        "search": {"cells": cells, "ms": 1e3 * s_sec, "cells_per_s": cells / s_sec, "zmax": zmax,
                   "numharm": numharm, "candidates": int(ncand),
                   "tuning": plan.tuning().strip().split("\n")},
        "end_to_end_ms": 1e3 * e_sec,
        "phases_ms": {k: round(v[0] / args.steps, 4) for k, v in ph.items()},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
