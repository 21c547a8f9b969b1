#!/usr/bin/env python3
"""Throughput of the densification hot path on one MI355X.

A step is one pass of the whole hot path over one batch of synthetic input:
edge-score maps of every view (grayscale, blur, Sobel, suppression, median
normalisation) followed by Long-Axis-Split of the selected Gaussians. The
default workload is the full densification step: 300 views of widths
1000-2473 (BF16 intermediate storage, every view in one launch per stage)
and LAS on 3M Gaussians with 20% selected, recorded once as a HIP graph and
replayed per step. The plain per-view FP32 form of the same step is timed
beside it, the dominant kernel is timed live with HIP events on its own
stream for the roofline, and the CPU oracle is timed on a bounded sample.

Prints one JSON line. Inputs are resident in HBM before timing starts. The
live Gaussian count is set back to N on the device before every step (one
8-byte device copy inside the timed region), so every step splits the same K
of the same N rows. The default warm-up (25 steps) outlasts the GPU's
ramp from idle: the first ten or so steps after an idle period run up to 15%
slower, then the step settles.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "edge-map megapixels/s + Gaussians split/s, batched-FP16 vs plain-FP32, % HBM peak"
HBM_PEAK_GBS = 8000.0
VALU_PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9   # CUs x SIMDs x lanes per cycle x clock (non-packed)
# Algorithmic work of the fused stencil: dynamic VALU lane-operations per
# output pixel of its steady-state loop (an interior strip with 4-pixel
# aligned stores), by storage precision -- what one pixel costs without the
# halo rows and columns every strip recomputes, its set-up or the histogram
# flush. Counted from the kernel's gfx950 code; a CPU test recompiles the
# kernel and checks these figures against it.
LOOP_LANE_OPS_PER_PX = {"fp32": 41.75, "fp16": 45.75, "bf16": 42.25}
COPY_CAL_BYTES = 1 << 30
STORE_BYTES = {"fp32": 4, "fp16": 2, "bf16": 2}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def percentile_ms(events_pairs):
    return float(np.mean([a.elapsed_time(b) for a, b in events_pairs]))


def copy_calibration(nbytes: int):
    """A plain copy of known size: reads and writes nbytes per launch, so the
    HBM counters of its dispatches calibrate FETCH_SIZE and WRITE_SIZE."""
    import torch

    src = torch.randint(0, 255, (nbytes,), dtype=torch.uint8, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": nbytes, "launches": 3}), flush=True)


def _csv_rows(path_glob: str):
    import csv
    import glob

    rows = []
    for f in sorted(glob.glob(path_glob, recursive=True)):
        with open(f, newline="") as fh:
            rows.extend(csv.DictReader(fh))
    return rows


def _counter_kib(rows, name_part: str, counter: str):
    """Mean per-dispatch value (KiB) of a counter over dispatches whose kernel
    name contains name_part, and the number of dispatches."""
    vals = [float(r["Counter_Value"]) for r in rows
            if name_part in r["Kernel_Name"] and r["Counter_Name"] == counter]
    return (sum(vals) / len(vals), len(vals)) if vals else (None, 0)


def kernel_part(name: str) -> str:
    """The part of the hot path a traced kernel belongs to."""
    parts = (("edge_fused", "edge: fused stencil"), ("edge_persistent", "edge: persistent form"),
             ("median_", "edge: median"), ("normalise", "edge: normalise"),
             ("uf_", "edge: unfused ablation"), ("las_", "Long-Axis-Split (and full record)"),
             ("sel_", "split mask"), ("copyBuffer", "runtime copy"), ("Fill", "torch fill"))
    for key, part in parts:
        if key in name:
            return part
    return "other"


def summarise_profile(d: str, copy_bytes: int):
    """Turn the rocprofv3 outputs under directory d (trace/, fetch/, write/,
    copy_fetch/, copy_write/ and bench.json, see the commands recorded in the
    summaries) into the two short summaries kept under profiles/."""
    res = json.loads(open(os.path.join(d, "bench.json")).read().strip().splitlines()[-1])
    kernel = res["roofline"]["kernel"]
    # the instantiation the timed form runs: <storage precision, wavefronts per work-group>
    prec_code = {"fp32": 0, "fp16": 1, "bf16": 2}[res["config"]["intermediate"]]
    nw = int(res["config"]["tile"].split("x")[1])
    sym = {"edge_fused": "edge_fused_kernel", "edge_persistent": "edge_persistent_kernel"}[kernel] + \
        f"<{prec_code}, {nw}>"
    stats = _csv_rows(os.path.join(d, "trace", "**", "*kernel_stats.csv"))
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    wl = res["config"]["workload"]
    tag = f"{kernel}_w{res['config']['views']}v_{res['config']['intermediate']}"
    bench_cmd = "python3 bench.py --steps 10 --warmup 25 --no-cpu-baseline --no-other-workloads"
    lines = [f"# Kernel trace: {wl}", "",
             "Command (repo root, TMPDIR=/tmp):", "",
             f"    rocprofv3 --kernel-trace --stats --output-format csv -d <dir>/trace -o t -- {bench_cmd}"
             " > <dir>/bench.json", "",
             f"Benchmark line of that run: form `{res['config']['form']}`, tile {res['config']['tile']}, "
             f"{res['ms_per_step']} ms/step; live HIP-event time of `{kernel}`: {res['stage_ms']['fused']} ms.", "",
             "The four other workloads are left out of profiled runs (`--no-other-workloads`): they run the same "
             "kernels at other sizes, and would mix into the averages below.", "",
             "Every kernel of the run (the bench times the graph-captured step, then each further form and row "
             "on its own: the plain per-view FP32 form is the many small launches), with the part of the hot "
             "path it belongs to:", "",
             "| Kernel | Part | Calls | Average (us) | Min (us) | Max (us) | Share |", "|---|---|---|---|---|---|---|"]
    total = sum(float(r["TotalDurationNs"]) for r in stats) or 1.0
    for r in sorted(stats, key=lambda r: -float(r["TotalDurationNs"]))[:40]:
        nm = r["Name"].replace("igsp::(anonymous namespace)::", "").split("(")[0].replace("void ", "")
        nm = nm if len(nm) < 70 else nm[:67] + "..."
        lines.append(f"| `{nm}` | {kernel_part(nm)} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | "
                     f"{100 * float(r['TotalDurationNs']) / total:.1f}% |")
    avg = [float(r["AverageNs"]) for r in stats if sym in r["Name"]]
    # the dispatches one by one: the first ones run while the clocks still
    # ramp up from idle, so the median is given beside the average
    durs = sorted(float(r["End_Timestamp"]) - float(r["Start_Timestamp"])
                  for r in _csv_rows(os.path.join(d, "trace", "**", "*kernel_trace.csv")) if sym in r["Kernel_Name"])
    if avg:
        med = f", median {durs[len(durs) // 2] / 1e6:.4f} ms over {len(durs)} dispatches" if durs else ""
        lines += ["", f"`{kernel}` average over the trace: {avg[0] / 1e6:.4f} ms{med}; the benchmark's live "
                      f"measurement: {res['stage_ms']['fused']} ms."]
    open(os.path.join(ROOT, "profiles", f"{tag}_kernel_trace.md"), "w").write("\n".join(lines) + "\n")

    fetch, nf = _counter_kib(_csv_rows(os.path.join(d, "fetch", "**", "*counter_collection.csv")), sym, "FETCH_SIZE")
    write, nw = _counter_kib(_csv_rows(os.path.join(d, "write", "**", "*counter_collection.csv")), sym, "WRITE_SIZE")
    cf, _ = _counter_kib(_csv_rows(os.path.join(d, "copy_fetch", "**", "*counter_collection.csv")), "copy",
                         "FETCH_SIZE")
    cw, _ = _counter_kib(_csv_rows(os.path.join(d, "copy_write", "**", "*counter_collection.csv")), "copy",
                         "WRITE_SIZE")
    valu, nv = _counter_kib(_csv_rows(os.path.join(d, "valu", "**", "*counter_collection.csv")), sym,
                            "SQ_INSTS_VALU")
    lds_rows = _csv_rows(os.path.join(d, "lds", "**", "*counter_collection.csv"))
    lds, nl = _counter_kib(lds_rows, sym, "SQ_INSTS_LDS")
    bank, _ = _counter_kib(lds_rows, sym, "SQ_LDS_BANK_CONFLICT")
    idx_active, _ = _counter_kib(lds_rows, sym, "SQ_LDS_IDX_ACTIVE")
    conflict_rate = bank / (idx_active - bank) if None not in (bank, idx_active) and idx_active > bank else None
    f_fetch = copy_bytes / (cf * 1024) if cf else None
    f_write = copy_bytes / (cw * 1024) if cw else None
    traffic = (fetch * 1024 * f_fetch + write * 1024 * f_write) if None not in (fetch, write, f_fetch, f_write) \
        else None
    pmc_cmd = "python3 bench.py --steps 2 --warmup 1 --no-cpu-baseline --no-plain --no-other-workloads --stage-reps 2"
    t = [f"kernel: {kernel}",
         f"kernel_source_sha256: {kernel_source_digest()}",
         f"workload: {wl}",
         f"precision: {res['config']['intermediate']}",
         f"tile: {res['config']['tile']}",
         f"fetch_kib_per_dispatch: {fetch} ({nf} dispatches)",
         f"write_kib_per_dispatch: {write} ({nw} dispatches)",
         f"copy_calibration_bytes: {copy_bytes}",
         f"copy_fetch_kib: {cf}", f"copy_write_kib: {cw}",
         f"fetch_scale: {f_fetch}", f"write_scale: {f_write}",
         f"traffic_bytes_per_launch: {traffic}",
         f"algorithmic_bytes_per_launch: {res['roofline']['bytes_per_launch']}",
         f"valu_insts_per_launch: {valu} ({nv} dispatches; SQ_INSTS_VALU, wave instructions)",
         f"lds_insts_per_launch: {lds} ({nl} dispatches; SQ_INSTS_LDS, wave instructions)",
         f"lds_bank_conflict_cycles_per_launch: {bank} (SQ_LDS_BANK_CONFLICT, cycles summed over CUs)",
         f"lds_idx_active_cycles_per_launch: {idx_active} (SQ_LDS_IDX_ACTIVE)",
         f"lds_bank_conflict_rate: {conflict_rate} (conflict cycles / conflict-free active cycles)",
         "",
         "  Commands (repo root, TMPDIR=/tmp), each pass in its own run:",
         f"    timeout -s KILL 120 rocprofv3 --pmc FETCH_SIZE --output-format csv -d <dir>/fetch -o p -- {pmc_cmd}",
         f"    timeout -s KILL 120 rocprofv3 --pmc WRITE_SIZE --output-format csv -d <dir>/write -o p -- {pmc_cmd}",
         f"    timeout -s KILL 60 rocprofv3 --pmc FETCH_SIZE --output-format csv -d <dir>/copy_fetch -o p -- "
         f"python3 bench.py --copy-calibration {copy_bytes}",
         f"    timeout -s KILL 60 rocprofv3 --pmc WRITE_SIZE --output-format csv -d <dir>/copy_write -o p -- "
         f"python3 bench.py --copy-calibration {copy_bytes}",
         f"    timeout -s KILL 120 rocprofv3 --pmc SQ_INSTS_VALU SQ_WAVES --output-format csv -d <dir>/valu -o p -- "
         f"{pmc_cmd}",
         f"    timeout -s KILL 120 rocprofv3 --pmc SQ_INSTS_LDS SQ_LDS_BANK_CONFLICT SQ_LDS_IDX_ACTIVE --output-format csv -d <dir>/lds "
         f"-o p -- {pmc_cmd}",
         "    python3 bench.py --summarise-profile <dir>",
         "  FETCH_SIZE / WRITE_SIZE are KiB per dispatch; each is scaled by copy_bytes / (1024 x what the same",
         "  counter reads for the plain copy of copy_bytes bytes). traffic = scaled fetch + scaled write."]
    # the other kernels of the step and of the split-mask row, from the same passes
    if None not in (f_fetch, f_write):
        fetch_rows = _csv_rows(os.path.join(d, "fetch", "**", "*counter_collection.csv"))
        write_rows = _csv_rows(os.path.join(d, "write", "**", "*counter_collection.csv"))
        npx = res["config"]["megapixels"] * 1e6
        alg = {f"normalise_kernel<{prec_code}>": npx * (STORE_BYTES[res["config"]["intermediate"]] + 4)}
        t += ["", "Other kernels, same passes and scaling (MB per dispatch; algorithmic bytes where the "
                  "benchmark states them per kernel). The plain split and the full-record split (feature rows and "
                  "moments) are separate kernels:", "",
              "| Kernel | Dispatches | Fetch | Write | Traffic | Algorithmic |", "|---|---|---|---|---|---|"]
        for k in (f"normalise_kernel<{prec_code}>", f"median_select_kernel<{prec_code}>", "las_count_kernel",
                  "las_scan_kernel", "las_split_kernel", "las_split_full_kernel", "sel_scatter_kernel",
                  "sel_compact_kernel",
                  "sel_hist_kernel", "sel_mask_kernel"):
            fv = [float(r["Counter_Value"]) * 1024 * f_fetch for r in fetch_rows
                  if k in r["Kernel_Name"] and r["Counter_Name"] == "FETCH_SIZE"]
            wv = [float(r["Counter_Value"]) * 1024 * f_write for r in write_rows
                  if k in r["Kernel_Name"] and r["Counter_Name"] == "WRITE_SIZE"]
            if not fv or len(fv) != len(wv):
                continue
            tv = [x + y for x, y in zip(fv, wv)]

            def span(v):  # one figure, or the range where dispatches differ (several rows of the bench)
                lo, hi = min(v) / 1e6, max(v) / 1e6
                return f"{lo:.1f}" if hi - lo <= max(0.05 * hi, 0.05) else f"{lo:.1f}-{hi:.1f}"
            a_b = f"{alg[k] / 1e6:.1f}" if k in alg else "-"
            t.append(f"| `{k}` | {len(fv)} | {span(fv)} | {span(wv)} | {span(tv)} | {a_b} |")
    open(os.path.join(ROOT, "profiles", f"{kernel}_hbm_traffic.txt"), "w").write("\n".join(t) + "\n")
    print(json.dumps({"kernel": kernel, "traffic_bytes_per_launch": traffic, "trace_avg_ms":
                      avg[0] / 1e6 if avg else None, "live_ms": res["stage_ms"]["fused"]}))


def las_touched_bytes(mask: np.ndarray, K: int) -> int:
    """Bytes of whole 128-byte lines the split moves: the mask, every line
    holding a selected parent row of each array (read; written back for the
    fields the split changes: means, log-scales, opacity), and the K
    contiguous child rows plus their indices. With 20% of the rows selected
    nearly every parent line is touched, so this approaches N x 44 read."""
    idx = np.nonzero(mask)[0].astype(np.int64)

    def lines(row_bytes):
        first = idx * row_bytes // 128
        last = (idx * row_bytes + row_bytes - 1) // 128
        return np.unique(np.concatenate([first, last])).size * 128

    parent = 2 * lines(12) + 2 * lines(12) + lines(16) + 2 * lines(4)   # means, log-scales, quats, opacity
    return int(mask.size + parent + K * (44 + 4))


def cpu_model() -> str:
    """The host CPU's model name (first entry of /proc/cpuinfo), or "unknown"."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def kernel_source_digest() -> str:
    """SHA-256 over the kernel sources and the host code that orders their
    work-groups: counters taken on other sources do not describe this build."""
    import hashlib

    h = hashlib.sha256()
    for name in ("edge_kernels.hip", "select_kernels.hip", "las_kernels.hip", "igsp_api.hip", "igsp_internal.h"):
        h.update(open(os.path.join(ROOT, "paper_2603_08661_amd", "csrc", name), "rb").read())
    return h.hexdigest()


def profile_facts(kernel: str, prec: str, workload: str, seg_rows: int, wg_waves: int) -> dict:
    """Counter facts (HBM bytes, VALU and LDS instructions, LDS bank-conflict
    cycles per launch) of the dominant kernel from the committed summary, or
    {} when that summary was taken on another kernel source, workload,
    storage precision or tile shape."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_hbm_traffic.txt")
    try:
        kv = {}
        for line in open(path):
            if ":" in line and not line.startswith(" "):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
        digest = kernel_source_digest()
        if (kv.get("kernel_source_sha256") != digest or kv.get("precision") != prec
                or kv.get("workload") != workload or kv.get("tile") != f"{seg_rows}x{wg_waves}"):
            return {}
    except OSError:
        return {}
    out = {}
    for key in ("traffic_bytes_per_launch", "valu_insts_per_launch", "lds_insts_per_launch",
                "lds_bank_conflict_cycles_per_launch"):
        try:
            out[key] = int(float(kv[key].split()[0]))
        except (KeyError, ValueError, IndexError):
            pass
    try:
        out["lds_bank_conflict_rate"] = round(float(kv["lds_bank_conflict_rate"].split()[0]), 4)
    except (KeyError, ValueError, IndexError):
        pass
    return out


def main():
    import synth

    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=25)
    ap.add_argument("--workload", default="step_views300_las3m", choices=sorted(synth.WORKLOADS))
    ap.add_argument("--precision", default=None, help="override the workload's intermediate storage")
    ap.add_argument("--seg-rows", type=int, default=0)
    ap.add_argument("--wg-waves", type=int, default=0)
    ap.add_argument("--no-plain", action="store_true", help="skip the plain per-view FP32 comparison")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-select", action="store_true",
                    help="skip the split-mask generation (edge scores onto Gaussians, threshold, budget)")
    ap.add_argument("--contrib-order", default="rows", choices=["rows", "spread"],
                    help="order of the synthetic pixel contributions of the split-mask line")
    ap.add_argument("--no-las-full", action="store_true",
                    help="skip the full-record split (48 features + Adam moments)")
    ap.add_argument("--no-unfused", action="store_true",
                    help="skip the unfused (one launch per step) form of the same batch")
    ap.add_argument("--cpu-seconds", type=float, default=10.0, help="target CPU time of the oracle sample")
    ap.add_argument("--stage-reps", type=int, default=10)
    ap.add_argument("--no-other-workloads", action="store_true",
                    help="skip the compact lines of the four other workloads (single views, the 200- and "
                         "150-view batches)")
    ap.add_argument("--tune", action="store_true",
                    help="run the autotuner on this batch first (default: the library's tuned table)")
    ap.add_argument("--form", default="batched", choices=["batched", "staged", "persistent"],
                    help="batched launch form (batched: the tuned table's choice, else staged)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES bytes three times (counter calibration)")
    ap.add_argument("--summarise-profile", default=None, metavar="DIR",
                    help="only summarise rocprofv3 outputs under DIR into profiles/")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.summarise_profile:
        summarise_profile(args.summarise_profile, COPY_CAL_BYTES)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; multi-GPU sharding is not built "
                                   "(views would shard with no exchange, see the design notes)",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch

    import paper_2603_08661_amd as igsp

    dev = torch.device("cuda:0")
    w = synth.workload(args.workload)
    prec = args.precision or w.precision
    t0 = time.time()
    vb = w.render()
    log(f"workload {args.workload}: {vb.n} views, {vb.pixels / 1e6:.1f} MPx rendered in {time.time() - t0:.1f}s")
    img = torch.from_numpy(np.concatenate([vb.rgb, np.zeros(16, np.uint8)])).to(dev)
    out = torch.zeros(vb.out_floats, dtype=torch.float32, device=dev)
    views = (vb.widths, vb.heights, vb.in_offset, vb.out_offset)
    mpx = vb.pixels / 1e6

    has_las = w.n_gauss > 0
    if has_las:
        g = w.gaussian_set()
        mk = w.split_mask()
        N0, K = w.n_gauss, w.n_split
        cap = N0 + K     # every split starts again from N0 (reset_count)
        G = {}
        for k in ("means", "log_scales", "quats", "opacity_logits"):
            a = getattr(g, k)
            G[k] = torch.zeros((cap,) + a.shape[1:], dtype=torch.float32, device=dev)
            G[k][:N0] = torch.from_numpy(a).to(dev)
        G["count"] = torch.tensor([N0], dtype=torch.int64, device=dev)
        n0_dev = torch.tensor([N0], dtype=torch.int64, device=dev)
        mask = torch.zeros(cap, dtype=torch.uint8, device=dev)
        mask[:N0] = torch.from_numpy(mk).to(dev)
        sidx = torch.zeros(cap, dtype=torch.int32, device=dev)
        status = torch.zeros(1, dtype=torch.int32, device=dev)
        log(f"LAS: N={N0} K={K} capacity={cap}")
    torch.cuda.synchronize()

    stream = torch.cuda.Stream()

    def edge(p, ev=None):
        igsp.edge_importance(img, views, out, precision=p, batched=bform, seg_rows=args.seg_rows,
                             wg_waves=args.wg_waves, stage_events=ev, stream=stream)

    def reset_count():
        # the split grows N in place; every step starts again from the workload's N
        with torch.cuda.stream(stream):
            G["count"].copy_(n0_dev)

    def las():
        reset_count()
        igsp.long_axis_split(G["means"], G["log_scales"], G["quats"], G["opacity_logits"], G["count"], mask,
                             sidx, status, stream=stream)

    def timed(fn, warm, reps):
        for _ in range(warm):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        w0 = time.perf_counter()
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - w0) * 1e3 / reps
        return e0.elapsed_time(e1) / reps, wall

    # ---- launch form and tile shape: explicit, the library default, or
    #      autotuned on this batch
    if args.tune and args.seg_rows == 0 and args.wg_waves == 0:
        t1 = time.time()
        igsp.edge_autotune(img, views, out, precision=prec, batched=args.form, stream=stream)
        torch.cuda.synchronize()
        log(f"autotuned in {time.time() - t1:.2f}s")
    bform, seg, wgw = igsp.edge_resolve(views, prec, args.form, args.seg_rows, args.wg_waves)
    log(f"form={bform} seg_rows={seg} wg_waves={wgw}")
    args.seg_rows, args.wg_waves = seg, wgw

    # ---- primary form: batched, reduced-precision storage, graph-captured step
    if w.graph:
        with torch.cuda.stream(stream):
            step = igsp.Step(img, views, out, G, mask, sidx, status, precision=prec, batched=bform,
                             seg_rows=args.seg_rows, wg_waves=args.wg_waves, stream=stream)
        def run_primary():
            reset_count()
            step.launch(stream)
        form = f"batched ({bform}) {prec} + LAS, one HIP graph per step"
    else:
        def run_primary():
            edge(prec)
            if has_las:
                las()
        form = f"batched ({bform}) {prec}" + (" + LAS" if has_las else "")
    ms, wall = timed(run_primary, args.warmup, args.steps)
    log(f"primary ({form}): {ms:.3f} ms/step (wall {wall:.3f})")
    if has_las:
        assert int(status.item()) == 0, "split reported a capacity error"

    # ---- live stage timing of the dominant kernel (same configuration, eager)
    pairs = {k: [] for k in ("fused", "select", "normalise", "edge")}
    for _ in range(args.stage_reps):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        for e in ev:            # torch creates the HIP event on its first record
            e.record(stream)
        edge(prec, ev)
        torch.cuda.synchronize()
        pairs["fused"].append((ev[0], ev[1]))
        pairs["select"].append((ev[1], ev[2]))
        pairs["normalise"].append((ev[2], ev[3]))
        pairs["edge"].append((ev[0], ev[3]))
    stage_ms = {k: percentile_ms(v) for k, v in pairs.items()}
    las_ms = None
    if has_las:
        las_ms, _ = timed(las, 1, args.stage_reps)
    sb = STORE_BYTES[prec]
    if bform == "persistent":     # one kernel: RGB in, maps out
        kernel, per_px = "edge_persistent", 7
    else:                         # the stencil kernel: RGB in, stored survivors out
        kernel, per_px = "edge_fused", 3 + sb
    fused_bytes = vb.pixels * per_px
    achieved = fused_bytes / (stage_ms["fused"] * 1e-3) / 1e9
    log(f"stages: {stage_ms}, las {las_ms}")

    # ---- which Gaussians to split: edge scores of this step's maps moved onto
    #      the Gaussians through synthetic pixel contributions, then the
    #      gradient threshold and the budget (N, K of the same workload)
    select = None
    if has_las and not args.no_select:
        t1 = time.time()
        cb = synth.contributions(7000001 * w.stream + 2, N0, vb.widths, vb.heights, 3, order=args.contrib_order)
        gr = synth.grad_accum(7000001 * w.stream + 3, N0)
        thr = float(np.quantile(gr, 0.6))          # 40% of the Gaussians pass the gradient test
        log(f"contributions: {cb.n} entries ({time.time() - t1:.1f}s)")
        T = lambda a: torch.from_numpy(a).to(dev)  # noqa: E731
        cg, cv, cp, cw, tg = T(cb.gauss), T(cb.view), T(cb.pixel), T(cb.weight), T(gr)
        smask = torch.zeros(N0, dtype=torch.uint8, device=dev)
        sscore = torch.zeros(N0, dtype=torch.int64, device=dev)
        scount = torch.tensor([N0], dtype=torch.int64, device=dev)
        snsel = torch.zeros(1, dtype=torch.int64, device=dev)

        def run_select():
            igsp.split_mask(out, views, cg, cv, cp, cw, tg, scount, smask, sscore, grad_threshold=thr,
                            budget=N0 + K, n_selected=snsel, stream=stream)
        sms, _ = timed(run_select, 1, 5)
        sbytes = 28 * cb.n + 133 * N0
        select = {"contributions": cb.n, "order": args.contrib_order, "gaussians": N0,
                  "selected": int(snsel.item()), "ms": round(sms, 4),
                  "contributions_per_s": round(cb.n / (sms * 1e-3), 1),
                  "algorithmic_bytes": int(sbytes), "algorithmic_GBps": round(sbytes / (sms * 1e-3) / 1e9, 1),
                  "frac_of_hbm_peak": round(sbytes / (sms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        log(f"split mask: {sms:.3f} ms, {select['selected']} selected")
        del cg, cv, cp, cw, tg, cb

    # ---- the full-record split a trainer calls: 48 feature floats per row
    #      and both Adam moments of every parameter group (same N, K, mask)
    las_full = None
    if has_las and not args.no_las_full:
        F = 48
        reps = 5
        capf = N0 + K * (reps + 1)
        widths = {"means": 3, "log_scales": 3, "quats": 4, "opacity_logits": 1, "features": F}
        Gf = {}
        for k in ("means", "log_scales", "quats", "opacity_logits"):
            a = getattr(g, k)
            Gf[k] = torch.zeros((capf,) + a.shape[1:], dtype=torch.float32, device=dev)
            Gf[k][:N0] = torch.from_numpy(a).to(dev)
        Gf["features"] = torch.randn((capf, F), dtype=torch.float32, device=dev)
        mom = {grp: tuple(torch.randn((capf, w) if w > 1 else (capf,), dtype=torch.float32, device=dev)
                          for _ in range(2)) for grp, w in widths.items()}
        cnt = torch.tensor([N0], dtype=torch.int64, device=dev)
        maskf = torch.zeros(capf, dtype=torch.uint8, device=dev)
        maskf[:N0] = torch.from_numpy(mk).to(dev)
        sidxf = torch.zeros(capf, dtype=torch.int32, device=dev)
        stf = torch.zeros(1, dtype=torch.int32, device=dev)

        def run_full():
            igsp.long_axis_split_full(Gf["means"], Gf["log_scales"], Gf["quats"], Gf["opacity_logits"], cnt,
                                      maskf, sidxf, stf, mom, features=Gf["features"], stream=stream)
        fms, _ = timed(run_full, 1, reps)
        assert int(stf.item()) == 0, "full-record split reported a capacity error"
        per_split = (44 + 4 * F) + (28 + 44 + 4 * F + 4) + 2 * 2 * 4 * sum(widths.values())
        fbytes = N0 + per_split * K
        las_full = {"feat_dim": F, "adam_moments": "m and v of all five groups", "ms": round(fms, 4),
                    "gaussians_split_per_s": round(K / (fms * 1e-3), 1),
                    "algorithmic_bytes": int(fbytes),
                    "algorithmic_GBps": round(fbytes / (fms * 1e-3) / 1e9, 1),
                    "frac_of_hbm_peak": round(fbytes / (fms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        log(f"full-record split: {fms:.3f} ms")
        del Gf, mom, maskf, sidxf

    # ---- the paper's unfused layout on the same batch and storage precision
    unfused = None
    if not args.no_unfused:
        def run_unfused():
            igsp.edge_importance(img, views, out, precision=prec, batched="unfused", stream=stream)
        ums, _ = timed(run_unfused, 1, max(1, min(args.steps, 5)))
        unfused = {"form": f"unfused batched {prec} (gray, blur, Sobel, suppression as separate launches)",
                   "edge_ms": round(ums, 4), "mpx_per_s": round(mpx / (ums * 1e-3), 1),
                   "fused_edge_speedup": round(ums / stage_ms["edge"], 3)}
        log(f"unfused edge maps: {ums:.3f} ms")
        igsp.release_plans()   # frees the unfused form's per-step buffers

    # ---- practical ceiling of a read+write stream: a plain device copy
    cbytes = 1 << 30
    csrc = torch.empty(cbytes, dtype=torch.uint8, device=dev)
    cdst = torch.empty_like(csrc)
    def copy_once():
        with torch.cuda.stream(stream):
            cdst.copy_(csrc)
    cms, _ = timed(copy_once, 2, 10)
    copy_gbps = 2 * cbytes / (cms * 1e-3) / 1e9
    del csrc, cdst

    # ---- plain per-view FP32 form of the same step
    plain = None
    if not args.no_plain:
        def run_plain():
            igsp.edge_importance(img, views, out, precision="fp32", batched=False, stream=stream)
            if has_las:
                las()
        pms, pwall = timed(run_plain, 1, max(1, min(args.steps, 5)))
        plain = {"form": "plain per-view fp32" + (" + LAS" if has_las else ""), "ms_per_step": round(pms, 4),
                 "mpx_per_s": round(mpx / (pms * 1e-3), 1)}
        if has_las:
            plain["gaussians_split_per_s"] = round(K / (pms * 1e-3), 1)
        log(f"plain fp32: {pms:.3f} ms/step")

    # ---- the other workloads, compact: each in its primary form beside the
    #      plain per-view FP32 form of the same views (and, for the two
    #      single views, their split); the 150-view batch in FP16 and BF16
    others = None
    acc_sample = []      # (workload, precision, view index, that view's map) for the accuracy check
    if not args.no_other_workloads:
        others = {}
        for name in ("view_256x192", "view_1297x840", "views200_w1000_1560", "views150_2473x1643_mixed"):
            ow = synth.workload(name)
            t1 = time.time()
            ovb = ow.render()
            oimg = torch.from_numpy(np.concatenate([ovb.rgb, np.zeros(16, np.uint8)])).to(dev)
            oout = torch.zeros(ovb.out_floats, dtype=torch.float32, device=dev)
            oviews = (ovb.widths, ovb.heights, ovb.in_offset, ovb.out_offset)
            ompx = ovb.pixels / 1e6
            single = ovb.n == 1
            reps = 200 if single else 10
            entry = {"workload": ow.name, "views": int(ovb.n), "megapixels": round(ompx, 3)}
            for p in ow.extra.get("precisions", [ow.precision]):
                form = "plain" if single else "batched"
                oform, oseg, owgw = igsp.edge_resolve(oviews, p, form, 0, 0)

                def run_edge(p=p, oform=oform):
                    igsp.edge_importance(oimg, oviews, oout, precision=p, batched=oform, stream=stream)
                # warm-up long enough for the clocks to ramp up again after
                # the host-side rendering of the workload
                ems, _ = timed(run_edge, 50 if single else 25, reps)
                r = {"form": f"{'plain per-view' if single else 'batched (' + oform + ')'} {p}",
                     "tile": f"{oseg}x{owgw}", "edge_ms": round(ems, 4), "mpx_per_s": round(ompx / (ems * 1e-3), 1)}
                if not single:
                    r["algorithmic_GBps"] = round(ovb.pixels * 7 / (ems * 1e-3) / 1e9, 1)
                    r["frac_of_hbm_peak"] = round(ovb.pixels * 7 / (ems * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
                if name == "views200_w1000_1560":
                    # the same batch as one persistent launch, beside the tuned form
                    def run_persist(p=p):
                        igsp.edge_importance(oimg, oviews, oout, precision=p, batched="persistent", stream=stream)
                    pms_, _ = timed(run_persist, 25, reps)
                    r["persistent_edge_ms"] = round(pms_, 4)
                    r["persistent_mpx_per_s"] = round(ompx / (pms_ * 1e-3), 1)
                entry[p] = r
                if name == "views150_2473x1643_mixed":
                    E = oout.cpu().numpy()
                    for v in (0, 1):
                        o, W_, H_ = int(ovb.out_offset[v]), int(ovb.widths[v]), int(ovb.heights[v])
                        acc_sample.append((name, p, v, ovb.view(v), E[o:o + W_ * H_].reshape(H_, W_).copy()))
            if not single:
                def run_plain32():
                    igsp.edge_importance(oimg, oviews, oout, precision="fp32", batched=False, stream=stream)
                pms, _ = timed(run_plain32, 1, 3)
                best = min(entry[p]["edge_ms"] for p in ow.extra.get("precisions", [ow.precision]))
                entry["plain_fp32"] = {"edge_ms": round(pms, 4), "mpx_per_s": round(ompx / (pms * 1e-3), 1)}
                entry["speedup_vs_plain_fp32"] = round(pms / best, 3)
            if ow.n_gauss > 0:
                og = ow.gaussian_set()
                omk = ow.split_mask()
                oN, oK = ow.n_gauss, ow.n_split
                # every call splits the same K of the same N rows: the live
                # count is set back to N on the device before each call (an
                # 8-byte copy, timed on its own and taken off the split's time)
                ocap = oN + oK
                OG = {}
                for k in ("means", "log_scales", "quats", "opacity_logits"):
                    a = getattr(og, k)
                    OG[k] = torch.zeros((ocap,) + a.shape[1:], dtype=torch.float32, device=dev)
                    OG[k][:oN] = torch.from_numpy(a).to(dev)
                ocnt = torch.tensor([oN], dtype=torch.int64, device=dev)
                on0 = torch.tensor([oN], dtype=torch.int64, device=dev)
                omask = torch.zeros(ocap, dtype=torch.uint8, device=dev)
                omask[:oN] = torch.from_numpy(omk).to(dev)
                osidx = torch.zeros(ocap, dtype=torch.int32, device=dev)
                ost = torch.zeros(1, dtype=torch.int32, device=dev)

                def run_reset():
                    with torch.cuda.stream(stream):
                        ocnt.copy_(on0)

                def run_split():
                    run_reset()
                    igsp.long_axis_split(OG["means"], OG["log_scales"], OG["quats"], OG["opacity_logits"], ocnt,
                                         omask, osidx, ost, stream=stream)
                rms, _ = timed(run_reset, 20, reps)
                lms, _ = timed(run_split, 20, reps)
                assert int(ost.item()) == 0, "split reported a capacity error"
                lms = max(lms - rms, 1e-6)
                entry["las"] = {"gaussians": oN, "split": oK, "ms": round(lms, 4), "count_reset_ms": round(rms, 4),
                                "gaussians_split_per_s": round(oK / (lms * 1e-3), 1)}
                del OG, omask, osidx
            del oimg, oout
            others[name] = entry
            log(f"workload {name}: {entry} ({time.time() - t1:.1f}s)")

    # ---- CPU oracle on a bounded sample
    cpu = None
    if not args.no_cpu_baseline:
        import oracle

        threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)
        v0 = vb.view(0)
        t1 = time.perf_counter()
        oracle.edge_view(v0)
        tv = time.perf_counter() - t1
        per_thread = max(1, int(round(args.cpu_seconds / max(tv, 1e-3) / 2)))
        nsamp = min(vb.n, threads * per_thread)
        sel = np.arange(nsamp)
        sub = synth.pack_views([vb.view(int(v)) for v in sel])
        t1 = time.perf_counter()
        oracle.edge_batch(sub.rgb, sub.widths, sub.heights, sub.in_offset, sub.out_offset, sub.out_floats,
                          threads=threads)
        te = time.perf_counter() - t1
        # the same oracle on one core, on a shorter prefix of the views
        per_view_1core = te * threads / max(nsamp, 1)
        n1 = max(1, min(nsamp, int(round(args.cpu_seconds / 2 / max(per_view_1core, 1e-3)))))
        sub1 = synth.pack_views([vb.view(v) for v in range(n1)])
        t1 = time.perf_counter()
        oracle.edge_batch(sub1.rgb, sub1.widths, sub1.heights, sub1.in_offset, sub1.out_offset, sub1.out_floats,
                          threads=1)
        t1c = time.perf_counter() - t1
        cpu = {"value": round(sub.pixels / 1e6 / te, 3), "unit": "MPx/s", "cores": threads, "kind": "oracle",
               "value_1core": round(sub1.pixels / 1e6 / t1c, 3), "cpu_model": cpu_model(),
               "sample": f"edge maps of the first {nsamp} views ({sub.pixels / 1e6:.1f} MPx) of the same "
                         f"workload, views spread over {threads} threads, {te:.1f}s; on 1 core the first "
                         f"{n1} views ({sub1.pixels / 1e6:.1f} MPx), {t1c:.1f}s"}
        if has_las:
            n_l = min(N0, 1_000_000)
            k_l = int(mk[:n_l].sum())
            h = {}
            for k in ("means", "log_scales", "quats", "opacity_logits"):
                a = getattr(g, k)
                h[k] = np.zeros((n_l + k_l,) + a.shape[1:], np.float32)
                h[k][:n_l] = a[:n_l]
            t1 = time.perf_counter()
            r = oracle.las(n_l, h["means"], h["log_scales"], h["quats"], h["opacity_logits"], mk[:n_l])
            tl = time.perf_counter() - t1
            cpu["gaussians_split_per_s"] = round(r["K"] / tl, 1) if r["status"] == 0 else None
            cpu["sample"] += f"; split of the first {n_l} Gaussians ({r['K']} selected) on 1 thread, {tl:.2f}s"
        log(f"cpu baseline: {cpu}")
        # The oracle's maps of the sampled views of the 150-view batch, against
        # the maps this run's GPU form wrote for them: suppression decisions
        # that differ (and how many of those the oracle's margin exempts), the
        # map error over equal decisions, scaled by max(1, E) and plain.
        refs = {}
        for name, p, v, rgb, Eg in acc_sample:
            if (name, v) not in refs:
                refs[(name, v)] = oracle.edge_view(rgb)
            ref = refs[(name, v)]
            keep_g, keep_r = Eg > 0, ref["keep"] > 0
            mism = keep_g != keep_r
            same = ~mism
            d = np.abs(Eg.astype(np.float64) - ref["E"])[same]
            a = others[name][p].setdefault("accuracy", {"views": [], "pixels": 0, "decisions_differing": 0,
                                                        "differing_not_exempt": 0, "max_scaled_err": 0.0,
                                                        "max_abs_err": 0.0})
            a["views"].append(v)
            a["pixels"] += int(Eg.size)
            a["decisions_differing"] += int(mism.sum())
            a["differing_not_exempt"] += int((mism & (ref["margin"] >= 1e-6)).sum())
            a["max_scaled_err"] = max(a["max_scaled_err"], float((d / np.maximum(1.0, ref["E"][same])).max()))
            a["max_abs_err"] = max(a["max_abs_err"], float(d.max()))
        for name, p, *_ in acc_sample:
            a = others[name][p]["accuracy"]
            a["mismatch_rate"] = a["decisions_differing"] / max(a["pixels"], 1)

    prof = profile_facts(kernel, prec, w.name, seg, wgw)
    traffic = prof.get("traffic_bytes_per_launch")
    hbm = {"achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 4), "algorithmic_bytes_per_px": per_px,
           "bytes_per_launch": int(fused_bytes)}
    if traffic:
        tg = traffic / (stage_ms["fused"] * 1e-3) / 1e9
        hbm["traffic_GBps"] = round(tg, 1)
        hbm["traffic_frac"] = round(tg / HBM_PEAK_GBS, 4)
    if kernel == "edge_fused":
        # bound by vector-ALU issue (counters: VALU busy ~85%, HBM ~43%):
        # algorithmic lane-operations per launch against the VALU peak
        ops = LOOP_LANE_OPS_PER_PX[prec] * vb.pixels
        alu = ops / (stage_ms["fused"] * 1e-3) / 1e12
        roof = {"bound": "alu", "kernel": kernel, "achieved": round(alu, 2),
                "peak": round(VALU_PEAK_LANE_OPS / 1e12, 2), "unit": "TOP/s",
                "frac": round(alu * 1e12 / VALU_PEAK_LANE_OPS, 4), "traffic": traffic,
                "algorithmic_lane_ops_per_px": LOOP_LANE_OPS_PER_PX[prec], "ops_per_launch": int(ops),
                "bytes_per_launch": int(fused_bytes), "hbm": hbm}
    else:
        roof = dict(hbm, bound="hbm", kernel=kernel, traffic=traffic)
    if prof.get("valu_insts_per_launch"):
        lane_ops = prof["valu_insts_per_launch"] * 64
        roof["valu_lane_ops_per_px"] = round(lane_ops / vb.pixels, 2)
        roof["valu_frac"] = round(lane_ops / (stage_ms["fused"] * 1e-3) / VALU_PEAK_LANE_OPS, 4)
    if prof.get("lds_insts_per_launch") is not None:
        roof["lds_insts_per_launch"] = prof["lds_insts_per_launch"]
    if prof.get("lds_bank_conflict_rate") is not None:
        roof["lds_bank_conflict_rate"] = prof["lds_bank_conflict_rate"]
    res = {
        "metric": METRIC,
        "value": round(mpx / (ms * 1e-3), 1),
        "unit": "MPx/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "views": vb.n, "megapixels": round(mpx, 2),
                   "intermediate": prec, "form": form, "gaussians": w.n_gauss, "split": w.n_split,
                   "tile": f"{seg}x{wgw}",
                   "arithmetic": "int32 exact through Sobel, fp32 magnitude/suppression/median/LAS"},
        "wall_ms_per_step": round(wall, 4),
        "stage_ms": {k: round(v, 4) for k, v in stage_ms.items()},
        "roofline": roof,
        "copy_ceiling_GBps": round(copy_gbps, 1),
        "normalise": {"ms": round(stage_ms["normalise"], 4),
                      "algorithmic_bytes": int(vb.pixels * (sb + 4)),
                      "algorithmic_GBps": round(vb.pixels * (sb + 4) / (stage_ms["normalise"] * 1e-3) / 1e9, 1),
                      "frac_of_hbm_peak": round(vb.pixels * (sb + 4) / (stage_ms["normalise"] * 1e-3) / 1e9
                                                / HBM_PEAK_GBS, 4)} if stage_ms.get("normalise", 0) > 0.01 else None,
        "edge_pipeline": {"ms": round(stage_ms["edge"], 4),
                          "mpx_per_s": round(mpx / (stage_ms["edge"] * 1e-3), 1),
                          "algorithmic_GBps": round(vb.pixels * 7 / (stage_ms["edge"] * 1e-3) / 1e9, 1),
                          "frac_of_hbm_peak": round(vb.pixels * 7 / (stage_ms["edge"] * 1e-3) / 1e9
                                                    / HBM_PEAK_GBS, 4)},
    }
    if has_las:
        res["gaussians_split_per_s"] = round(K / (ms * 1e-3), 1)
        las_bytes = N0 + 120 * K
        touched = las_touched_bytes(mk[:N0], K)
        res["las"] = {"ms": round(las_ms, 4), "gaussians_split_per_s": round(K / (las_ms * 1e-3), 1),
                      "algorithmic_bytes": int(las_bytes),
                      "algorithmic_GBps": round(las_bytes / (las_ms * 1e-3) / 1e9, 1),
                      "touched_bytes": int(touched),
                      "touched_GBps": round(touched / (las_ms * 1e-3) / 1e9, 1),
                      "frac_of_hbm_peak": round(las_bytes / (las_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                      "touched_frac_of_hbm_peak": round(touched / (las_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    if select:
        res["split_mask"] = select
    if las_full:
        res["las_full_record"] = las_full
    if unfused:
        res["unfused"] = unfused
    if others:
        res["other_workloads"] = others
    if plain:
        res["plain_fp32"] = plain
        res["speedup_vs_plain_fp32"] = round(plain["ms_per_step"] / ms, 3)
    if cpu:
        res["cpu_baseline"] = cpu
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
