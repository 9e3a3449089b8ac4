"""Benchmark of the fast Haar transform on one MI355X.

One step = the whole hot path on one synthetic input: the 5-level separable
2D analysis of a 4096 x 4096 FP32 smooth image followed by its synthesis
(fwd + inv).  Throughput is effective bandwidth: the algorithmic bytes of a
step (each direction reads its input once and writes its output once,
4 * N * 4 bytes) divided by the step time.  Inputs are resident in HBM; 16
buffer sets rotate so that the data of a step was last touched 15 steps
earlier.  The steps are independent, so they are issued round-robin on two
streams (each step's synthesis after its own analysis): the ramp-up and the
tail of one kernel then overlap another step's kernel, as in any stream of
independent transforms; the single-stream figure is reported beside it.  Many sets are needed because the kernels store with nontemporal
hints: their outputs never enter the 256 MB Infinity Cache, so only reads
evict it, and with few sets a step's input is still cached from its last use.

Printed: one JSON line with the contract fields, a ``roofline`` object for
the dominant kernel (timed per launch with HIP events on the launch stream),
the autograd fwd+bwd throughput at the same shape, and a ``cpu_baseline``
object (the FP64 oracle on a bounded sample, on this host's cores).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "effective GB/s & % HBM peak, Haar fwd+inv 2D 4096² 5-level; fwd+bwd vs plain"
H = W = 4096
LEVELS = 5
PEAK_GBPS = 8000.0          # MI355X HBM3E, 8 TB/s
SETS = 16
NSTREAMS = 2                # independent steps alternate between this many streams
# the code of the timed launches: their kernels and the host code that picks
# their tile shape, load hints and block order
KERNEL_SOURCES = ["paper_1002_2184_amd/csrc/haar_2d.hip", "paper_1002_2184_amd/csrc/haar_2d_tile.h",
                  "paper_1002_2184_amd/csrc/haar_device.h", "paper_1002_2184_amd/csrc/haar_api.hip",
                  "paper_1002_2184_amd/csrc/haar_tune.hip"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_fwd2d_inv2d_4096x4096_L5.json")


def _code_only(text: str) -> str:
    """Source text without comments and blank lines: edits to comments do not
    change the kernels, so they do not invalidate a traffic measurement."""
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    lines = (re.sub(r"//.*$", "", ln).rstrip() for ln in text.splitlines())
    return "\n".join(ln for ln in lines if ln.strip())


def kernel_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), encoding="utf-8") as f:
            h.update(_code_only(f.read()).encode())
    return h.hexdigest()[:16]


def load_traffic(kernel: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or None
    when there is none or the kernel sources changed since it was taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_sources_sha256_16") != kernel_hash():
        return None
    entry = t.get("kernels", {}).get(kernel)
    return None if entry is None else entry.get("hbm_bytes_per_launch")


def pmc_probe():
    """Dispatches for rocprofv3 counter passes: a plain 64 MiB device copy (the
    calibration reference of known size), then the fwd2d and inv2d kernels of
    the benchmark workload, 8 of each, on rotating buffers."""
    import torch
    from paper_1002_2184_amd import transform as T
    from workloads import generators as G
    dev = torch.device("cuda", 0)
    x0 = torch.from_numpy(G.config2(H, W)).to(dev)
    xs = [x0.clone() for _ in range(SETS)]
    ys = [torch.empty_like(x0) for _ in range(SETS)]
    zs = [torch.empty_like(x0) for _ in range(SETS)]
    for k in range(8):
        ys[k % SETS].copy_(xs[k % SETS])
    torch.cuda.synchronize()
    for k in range(8):
        s = k % SETS
        T.fwd2d(xs[s], LEVELS, out=ys[s])
        T.inv2d(ys[s], LEVELS, out=zs[s])
    torch.cuda.synchronize()
    print("pmc probe done", flush=True)


def write_traffic(fetch_csv: str, write_csv: str, command: str):
    """Turn two rocprofv3 --pmc counter CSVs (FETCH_SIZE, WRITE_SIZE; KiB per
    dispatch) into HBM bytes per launch of fwd2d / inv2d, each counter scaled
    by what it reads for the 64 MiB reference copy, and write the committed
    summary (JSON for bench.py, Markdown for people)."""
    import csv
    import statistics

    def per_kernel(path, counter):
        out = {}
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] != counter:
                continue
            name = r["Kernel_Name"]
            key = ("copy" if "copyBuffer" in name or "copy_kernel" in name else
                   "fwd2d" if "fwd2d_kernel" in name else "inv2d" if "inv2d_kernel" in name else None)
            if key:
                out.setdefault(key, []).append(float(r["Counter_Value"]))
        return {k: statistics.median(v) for k, v in out.items()}

    fetch = per_kernel(fetch_csv, "FETCH_SIZE")
    write = per_kernel(write_csv, "WRITE_SIZE")
    ref_kib = H * W * 4 / 1024.0
    f_scale, w_scale = ref_kib / fetch["copy"], ref_kib / write["copy"]
    alg = 2 * H * W * 4
    kernels = {}
    for k in ("fwd2d", "inv2d"):
        rd = fetch[k] * f_scale * 1024.0
        wr = write[k] * w_scale * 1024.0
        kernels[k] = {"fetch_kib_raw": fetch[k], "write_kib_raw": write[k],
                      "hbm_read_bytes": int(rd), "hbm_write_bytes": int(wr),
                      "hbm_bytes_per_launch": int(rd + wr),
                      "vs_algorithmic": round((rd + wr) / alg, 4)}
    doc = {"workload": "2d-smooth-4096x4096-L5", "command": command,
           "reference": {"kernel": "torch copy_ of 64 MiB (hipMemcpy device-to-device)",
                         "fetch_kib_raw": fetch["copy"], "write_kib_raw": write["copy"],
                         "fetch_scale": round(f_scale, 5), "write_scale": round(w_scale, 5)},
           "algorithmic_bytes_per_launch": alg,
           "kernel_sources_sha256_16": kernel_hash(), "kernels": kernels}
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(doc, f, indent=1)
    md = TRAFFIC_FILE[:-5] + ".md"
    with open(md, "w") as f:
        f.write(f"# HBM traffic per launch, 4096x4096 FP32, 5 levels\n\nCommand: `{command}`\n\n")
        f.write(f"Reference: 64 MiB device copy reads FETCH_SIZE = {fetch['copy']:.0f} KiB "
                f"(scale {f_scale:.4f}) and WRITE_SIZE = {write['copy']:.0f} KiB (scale {w_scale:.4f}).\n\n")
        f.write("| kernel | FETCH_SIZE KiB | WRITE_SIZE KiB | HBM read MiB | HBM write MiB | total / algorithmic |\n")
        f.write("|---|---|---|---|---|---|\n")
        for k, v in kernels.items():
            f.write(f"| {k} | {v['fetch_kib_raw']:.0f} | {v['write_kib_raw']:.0f} | "
                    f"{v['hbm_read_bytes'] / 2**20:.2f} | {v['hbm_write_bytes'] / 2**20:.2f} | "
                    f"{v['vs_algorithmic']:.4f} |\n")
        f.write(f"\nKernel sources sha256[:16] = {kernel_hash()}, over the code without comments "
                f"(bench.py reports traffic only while the code matches).\n")
    print(json.dumps(doc))


# Counter probes of the other workloads: (kind) -> what the probe dispatches.
PMC_KINDS = {
    "bf16_4096": "fwd2d / inv2d kernels, 4096x4096 BF16, 5 levels, 16 rotating sets",
    "plans_cfg5": "2D plans of the 512 uneven images, 4 levels, fwd and bwd, in BF16 and in FP32",
    "plans_cfg3": "1D plans of the 1024 uneven sine-mix signals, full depth, fwd and inv, FP32",
    "fused": "fused one-pass kernels, FP32: soft shrinkage of the 4096x4096 image (L5) and of "
             "256 x 65536 signals (L12), the sparsity-loss training step on 192 x 512^2 (L3)",
    "volumes": "3D kernels on the 4 x 256^3 phantom volumes, 3 levels, fwd and inv, FP32 and BF16",
}


# raw profiler output (counter CSVs, per-kind algorithmic bytes) lives in
# this folder of the repository, beside the rocprofv3 output directories
RAW_DIR = os.path.join(ROOT, "gpurun_out")


def _alg_file(kind: str) -> str:
    return os.path.join(RAW_DIR, f"pmc_{kind}_alg.json")


def pmc_probe_kind(kind: str):
    """Dispatches for the counter passes of one of PMC_KINDS: a 64 MiB device
    copy (the calibration reference), then 4 launches of each kernel of the
    workload.  Writes the algorithmic bytes of one dispatch of each kernel
    class to pmc_<kind>_alg.json in the raw-output folder for the summary."""
    import numpy as np
    import torch
    from paper_1002_2184_amd import plan as PL
    from paper_1002_2184_amd import transform as T
    from workloads import generators as G
    dev = torch.device("cuda", 0)
    ref = torch.empty(H * W, dtype=torch.float32, device=dev)
    ref2 = torch.empty_like(ref)
    for _ in range(4):
        ref2.copy_(ref)
    torch.cuda.synchronize()
    alg = {}
    if kind == "bf16_4096":
        x0 = torch.from_numpy(G.config2(H, W)).to(dev).to(torch.bfloat16)
        xs = [x0.clone() for _ in range(SETS)]
        ys = [torch.empty_like(x0) for _ in range(SETS)]
        zs = [torch.empty_like(x0) for _ in range(SETS)]
        for k in range(4):
            T.fwd2d(xs[k], LEVELS, out=ys[k])
            T.inv2d(ys[k], LEVELS, out=zs[k])
        alg = {"fwd2d bf16": 2 * H * W * 2, "inv2d bf16": 2 * H * W * 2}
    elif kind == "plans_cfg5":
        imgs, grads = G.config5()
        for name, dt in (("bf16", torch.bfloat16), ("f32", torch.float32)):
            if dt == torch.bfloat16:
                xs = [torch.from_numpy(a.view(np.int16)).to(dev).view(torch.bfloat16) for a in imgs]
                gs = [torch.from_numpy(a.view(np.int16)).to(dev).view(torch.bfloat16) for a in grads]
            else:
                xs = [torch.from_numpy(G.bf16_bits_to_f32(a)).to(dev) for a in imgs]
                gs = [torch.from_numpy(G.bf16_bits_to_f32(a)).to(dev) for a in grads]
            ys = [torch.empty_like(v) for v in xs]
            zs = [torch.empty_like(v) for v in gs]
            pf = PL.Plan2D(xs, ys, 4)
            pb = PL.Plan2D(gs, zs, 4, inverse=True)
            for _ in range(4):
                pf.execute()
                pb.execute()
            torch.cuda.synchronize()
            nb = 2 * sum(v.numel() for v in xs) * xs[0].element_size()
            alg[f"plan2d fwd {name}"] = nb
            alg[f"plan2d inv {name}"] = nb
            del xs, gs, ys, zs, pf, pb
            torch.cuda.empty_cache()
    elif kind == "plans_cfg3":
        sigs = G.config3()
        levels = [int(np.log2(v.size)) for v in sigs]
        xs = [torch.from_numpy(v).to(dev) for v in sigs]
        ys = [torch.empty_like(v) for v in xs]
        zs = [torch.empty_like(v) for v in xs]
        pf = PL.Plan1D(xs, ys, levels)
        pi = PL.Plan1D(ys, zs, levels, inverse=True)
        for _ in range(4):
            pf.execute()
            pi.execute()
        nb = 2 * sum(v.numel() for v in xs) * 4
        alg = {"plan1d fwd f32": nb, "plan1d inv f32": nb,
               "finish1d f32": 0}
    elif kind == "fused":
        x0 = torch.from_numpy(G.config2(H, W)).to(dev)
        xs = [x0.clone() for _ in range(4)]
        ys = [torch.empty_like(x0) for _ in range(4)]
        for k in range(4):
            T.shrink2d(xs[k], 5, [40.0, 20.0, 10.0, 5.0, 2.5], "soft", out=ys[k])
        del xs, ys
        x1 = [torch.randn(256, 65536, device=dev) for _ in range(4)]
        y1 = [torch.empty_like(v) for v in x1]
        for k in range(4):
            T.shrink1d(x1[k], 12, 0.5, "soft", out=y1[k])
        del x1, y1
        xa = [torch.randn(64 * 3, 512, 512, device=dev) for _ in range(2)]
        ga = [torch.empty_like(v) for v in xa]
        for k in range(4):
            T.l1_grad2d(xa[k % 2], 3, out=ga[k % 2])
        alg = {"shrink2d f32": 2 * H * W * 4, "shrink1d f32": 2 * 256 * 65536 * 4,
               "l1grad2d f32": 2 * 64 * 3 * 512 * 512 * 4, "l1 loss reduce": 0}
        del xa, ga
    elif kind == "volumes":
        vol = torch.from_numpy(G.to_storage(G.phantom_volume(G.rng_for(8), 256, 256, 256), G.F32)).to(dev)
        for name, dt in (("f32", torch.float32), ("bf16", torch.bfloat16)):
            vs = [vol.expand(4, 256, 256, 256).contiguous().to(dt) for _ in range(2)]
            cs = [torch.empty_like(v) for v in vs]
            for k in range(4):
                T.fwd3d(vs[k % 2], 3, out=cs[k % 2])
            for k in range(4):
                T.inv3d(cs[k % 2], 3, out=vs[(k + 1) % 2])
            nb = 2 * vs[0].numel() * vs[0].element_size()
            alg[f"fwd3d {name}"] = nb
            alg[f"inv3d {name}"] = nb
            del vs, cs
            torch.cuda.empty_cache()
    else:
        raise SystemExit(f"unknown counter probe {kind!r}; one of {sorted(PMC_KINDS)}")
    torch.cuda.synchronize()
    os.makedirs(os.path.dirname(_alg_file(kind)), exist_ok=True)
    with open(_alg_file(kind), "w") as f:
        json.dump(alg, f)
    print(f"pmc probe {kind} done", flush=True)


def _kernel_class(name: str):
    """Class of a dispatched kernel for the counter summaries, from its
    demangled name: the calibration copy, or '<kernel> <fwd|inv> <dtype>'."""
    if "copyBuffer" in name or "copy_kernel" in name:
        return "copy"
    dts = {"StF32": "f32", "StBF16": "bf16", "StF16": "f16"}

    def dtype_of(args):
        for k, v in dts.items():
            if k in args:
                return v
        return "?"
    m = re.search(r"plan2d_kernel<([^>]*)>", name)
    if m:
        a = [x.strip() for x in m.group(1).split(",")]
        return f"plan2d {'inv' if a[3] == 'true' else 'fwd'} {dtype_of(m.group(1))}"
    m = re.search(r"plan1d_kernel<([^>]*)>", name)
    if m:
        a = [x.strip() for x in m.group(1).split(",")]
        return f"plan1d {'inv' if a[1] == 'true' else 'fwd'} {dtype_of(m.group(1))}"
    m = re.search(r"(finish1d\w*|plan1d_finish_kernel)<([^>]*)>", name)
    if m:
        return f"finish1d {dtype_of(m.group(2))}"
    m = re.search(r"shrink2d_\w*kernel<([^>]*)>", name)
    if m:
        a = [x.strip() for x in m.group(1).split(",")]
        return f"{'l1grad2d' if a[3] == '1' else 'shrink2d'} {dtype_of(m.group(1))}"
    m = re.search(r"shrink1d_\w*kernel<([^>]*)>", name)
    if m:
        return f"shrink1d {dtype_of(m.group(1))}"
    if "l1_loss_reduce_kernel" in name:
        return "l1 loss reduce"
    for k in ("fwd3d", "inv3d"):
        m = re.search(k + r"_\w*kernel<([^>]*)>", name)
        if m:
            return f"{k} {dtype_of(m.group(1))}"
    for k in ("fwd2d", "inv2d"):
        m = re.search(k + r"\w*kernel<([^>]*)>", name)
        if m:
            return f"{k} {dtype_of(m.group(1))}"
    return None


def write_traffic_kind(kind: str, fetch_csv: str, write_csv: str, command: str, out_md: str):
    """Summarise the two counter passes of pmc_probe_kind into HBM bytes per
    dispatch of each kernel class, scaled by what the same counter reads for
    the 64 MiB reference copy, against the algorithmic bytes."""
    import csv
    import statistics
    with open(_alg_file(kind)) as f:
        alg = json.load(f)

    def per_class(path, counter):
        out, copies = {}, []
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] != counter:
                continue
            c = _kernel_class(r["Kernel_Name"])
            if c == "copy":      # the reference copies are the probe's first 4 dispatches
                copies.append((int(r["Dispatch_Id"]), float(r["Counter_Value"])))
            elif c is not None:
                out.setdefault(c, []).append(float(r["Counter_Value"]))
        res = {k: (statistics.median(v), len(v)) for k, v in out.items()}
        ref = [v for _, v in sorted(copies)[:4]]
        res["copy"] = (statistics.median(ref), len(ref))
        return res

    fetch = per_class(fetch_csv, "FETCH_SIZE")
    write = per_class(write_csv, "WRITE_SIZE")
    ref_kib = H * W * 4 / 1024.0
    f_scale, w_scale = ref_kib / fetch["copy"][0], ref_kib / write["copy"][0]
    with open(out_md, "w") as f:
        f.write(f"# HBM traffic per dispatch: {PMC_KINDS[kind]}\n\nCommand: `{command}`\n\n")
        f.write(f"Reference: a 64 MiB device copy reads FETCH_SIZE = {fetch['copy'][0]:.0f} KiB "
                f"(scale {f_scale:.4f}) and WRITE_SIZE = {write['copy'][0]:.0f} KiB (scale {w_scale:.4f}); "
                "each kernel's counters are scaled by the same factor.  Medians over the dispatches.\n\n")
        f.write("| kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | HBM read MiB | HBM write MiB "
                "| algorithmic MiB | total / algorithmic |\n|---|---|---|---|---|---|---|---|\n")
        for k in sorted(set(fetch) | set(write)):
            if k == "copy":
                continue
            fr, n = fetch.get(k, (0.0, 0))
            wr, _ = write.get(k, (0.0, 0))
            rd, wb = fr * f_scale * 1024.0, wr * w_scale * 1024.0
            a = alg.get(k)
            ratio = f"{(rd + wb) / a:.4f}" if a else "n/a (small)"
            am = f"{a / 2**20:.2f}" if a is not None else "?"
            f.write(f"| {k} | {n} | {fr:.0f} | {wr:.0f} | {rd / 2**20:.2f} | {wb / 2**20:.2f} | {am} | {ratio} |\n")
    print(open(out_md).read())


def _isolated_averages(trace_csv: str):
    """Per kernel name: (dispatches that overlapped no other dispatch, their
    average duration in us), from a rocprofv3 kernel-trace CSV.  Kernels that
    ran concurrently on other streams share the device, so only isolated
    dispatches give the kernel's own duration."""
    import csv
    rows = [(int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r["Kernel_Name"])
            for r in csv.DictReader(open(trace_csv))]
    rows.sort()
    out = {}
    end_max = -1
    for i, (a, b, name) in enumerate(rows):
        nxt = rows[i + 1][0] if i + 1 < len(rows) else None
        alone = a >= end_max and (nxt is None or nxt >= b)
        end_max = max(end_max, b)
        if alone:
            n, t = out.get(name, (0, 0.0))
            out[name] = (n + 1, t + (b - a) / 1e3)
    return {k: (n, t / n) for k, (n, t) in out.items()}


def write_kernel_stats(stats_csv: str, command: str, out_md: str, max_rows: int = 30):
    """Summarise a rocprofv3 --kernel-trace --stats CSV (one row per kernel
    name) into a short Markdown table under profiles/; with the kernel-trace
    CSV beside it, also the average over the dispatches that ran alone."""
    import csv
    rows = list(csv.DictReader(open(stats_csv)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    total = len(rows)
    rows = rows[:max_rows]
    trace = stats_csv[:-len("_kernel_stats.csv")] + "_kernel_trace.csv" \
        if stats_csv.endswith("_kernel_stats.csv") else None
    iso = _isolated_averages(trace) if trace and os.path.exists(trace) else {}
    with open(out_md, "w") as f:
        f.write(f"# Kernel durations (rocprofv3 --kernel-trace --stats)\n\nCommand: `{command}`\n\n")
        if total > len(rows):
            f.write(f"The {len(rows)} kernels with the most GPU time, of {total}.\n\n")
        if iso:
            f.write("`alone`: dispatches that overlapped no other dispatch (the benchmark also runs "
                    "steps on two streams at once, whose kernels share the device), and their average.\n\n")
        f.write("| kernel | calls | average us | min us | max us | share of GPU time | alone | average alone us |\n"
                "|---|---|---|---|---|---|---|---|\n")
        for r in rows:
            name = r["Name"]
            short = name if len(name) <= 110 else name[:107] + "..."
            n_iso, t_iso = iso.get(name, (0, 0.0))
            f.write(f"| `{short}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                    f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} | "
                    f"{float(r['Percentage']):.1f} % | {n_iso} | "
                    f"{(f'{t_iso:.2f}' if n_iso else '-')} |\n")
    print(open(out_md).read())


def _timed(fn, reps, warm, stream):
    import torch
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(reps):
        fn()
    b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def _graphed(fn, stream):
    """fn captured once into a HIP graph (after one eager warm-up on a side
    stream); returns the replay callable."""
    import torch
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(stream)
    with torch.cuda.stream(side):
        fn()
        with torch.cuda.graph(g, stream=side):
            fn()
    stream.wait_stream(side)
    torch.cuda.synchronize()
    return g.replay


def suite():
    """The other workloads, each beside the plain FP32 transform on this GPU.
    Prints one JSON line per workload (not the benchmark contract line)."""
    import numpy as np
    import torch

    from paper_1002_2184_amd import autograd as AG
    from paper_1002_2184_amd import plan as PL
    from paper_1002_2184_amd import transform as T
    from workloads import generators as G

    dev = torch.device("cuda", 0)
    st = torch.cuda.current_stream(dev)

    # 1) one 65536-sample FP32 signal, 16 levels: latency of fwd + inv
    x = torch.from_numpy(G.config1()).to(dev)
    y, z = torch.empty_like(x), torch.empty_like(x)

    def one():
        T.fwd1d(x, 16, out=y)
        T.inv1d(y, 16, out=z)
    ms = _timed(one, 200, 20, st)
    # 16 fwd+inv per graph: one replay of a two-kernel graph would mostly
    # time the graph launch itself
    g = torch.cuda.CUDAGraph()
    s2 = torch.cuda.Stream()
    s2.wait_stream(st)
    with torch.cuda.stream(s2):
        one()
        with torch.cuda.graph(g, stream=s2):
            for _ in range(16):
                one()
    st.wait_stream(s2)
    torch.cuda.synchronize()
    msg = _timed(g.replay, 20, 4, st) / 16
    print(json.dumps({"workload": "1d-white-65536-L16 fwd+inv", "us_eager": round(ms * 1e3, 2),
                      "us_graph": round(msg * 1e3, 2),
                      "gbps_eager": round(4 * 65536 * 4 / (ms * 1e-3) / 1e9, 1),
                      "note": "latency-bound: 1 MiB moved per fwd+inv"}), flush=True)

    # 2) 1024 uneven signals 2^10..2^20, full depth: one persistent launch
    sigs = G.config3()
    levels = [int(np.log2(v.size)) for v in sigs]
    xs = [torch.from_numpy(v).to(dev) for v in sigs]
    ys = [torch.empty_like(v) for v in xs]
    total = sum(v.numel() for v in xs)
    plan = PL.Plan1D(xs, ys, levels)
    ms_plan = _timed(plan.execute, 20, 3, st)
    ms_plan_graph = _timed(_graphed(plan.execute, st), 20, 3, st)

    def loop():
        for v, w, lv in zip(xs, ys, levels):
            T.fwd1d(v, lv, out=w)
    ms_loop = _timed(loop, 3, 1, st)
    flat = torch.cat([v.view(-1) for v in xs])[: (total // 65536) * 65536].view(-1, 65536)
    flat_y = torch.empty_like(flat)
    ms_plain = _timed(lambda: T.fwd1d(flat, 16, out=flat_y), 20, 3, st)
    print(json.dumps({"workload": "1d-batched-uneven-1024x2^[10,20]-fulldepth fwd",
                      "elements": int(total), "ms_plan": round(ms_plan, 4),
                      "gbps_plan": round(2 * total * 4 / (ms_plan * 1e-3) / 1e9, 1),
                      "ms_plan_graph": round(ms_plan_graph, 4),
                      "gbps_plan_graph": round(2 * total * 4 / (ms_plan_graph * 1e-3) / 1e9, 1),
                      "ms_per_signal_loop": round(ms_loop, 3),
                      "gbps_plain_same_bytes_65536x16": round(2 * flat.numel() * 4 / (ms_plain * 1e-3) / 1e9, 1)}),
          flush=True)
    del xs, ys, plan, flat, flat_y
    torch.cuda.empty_cache()

    # 3) autograd 64x3x512x512, 3 levels: fwd + bwd vs plain fwd + inv
    xa = torch.from_numpy(G.config4()).to(dev).requires_grad_(True)
    ga = torch.randn_like(xa)
    ya, za = torch.empty_like(xa), torch.empty_like(xa)
    n4 = xa.numel()

    def ag():
        out = AG.HaarFwd2D.apply(xa, 3)
        torch.autograd.grad(out, xa, ga)
    ms_ag = _timed(ag, 20, 3, st)
    xd = xa.detach()

    def plain():
        T.fwd2d(xd, 3, out=ya)
        T.inv2d(ya, 3, out=za)
    ms_pl = _timed(plain, 20, 3, st)
    print(json.dumps({"workload": "2d-autograd-64x3x512x512-L3 fwd+bwd",
                      "gbps_fwd_bwd": round(4 * n4 * 4 / (ms_ag * 1e-3) / 1e9, 1),
                      "gbps_plain_fwd_inv": round(4 * n4 * 4 / (ms_pl * 1e-3) / 1e9, 1),
                      "ms_fwd_bwd": round(ms_ag, 4), "ms_plain": round(ms_pl, 4)}), flush=True)

    # 3b) the whole training step of the sparsity loss sum|details| +
    #     0.5||LL_3||^2: autograd with the loss in torch, against the fused
    #     one-pass kernel (loss and gradient)
    ll_mask = torch.zeros(512, 512, dtype=torch.bool, device=dev)
    ll_mask[:64, :64] = True
    det_mask = ~ll_mask

    def step_unfused():
        y = AG.HaarFwd2D.apply(xa, 3)
        loss = (y.abs() * det_mask).sum() + 0.5 * (y * y * ll_mask).sum()
        torch.autograd.grad(loss, xa)
    ms_un = _timed(step_unfused, 10, 2, st)

    def step_fused():
        T.l1_grad2d(xd, 3, out=za)
    ms_fu = _timed(step_fused, 20, 3, st)
    print(json.dumps({"workload": "2d-64x3x512x512-L3 sparsity-loss training step (loss + grad)",
                      "ms_autograd_torch_loss": round(ms_un, 4), "ms_fused": round(ms_fu, 4),
                      "gbps_fused_one_pass": round(2 * n4 * 4 / (ms_fu * 1e-3) / 1e9, 1),
                      "speedup": round(ms_un / ms_fu, 2)}), flush=True)
    del xa, ga, ya, za, xd
    torch.cuda.empty_cache()

    # 4) 512 BF16 images, even H, W in [256, 2048], 4 levels: fwd + bwd plans,
    #    and the same images in FP32 through the same path
    imgs, grads = G.config5()
    res = {"workload": "2d-batched-bf16-512-uneven-L4 fwd+bwd"}
    for name, dt in (("bf16", torch.bfloat16), ("f32", torch.float32)):
        if dt == torch.bfloat16:
            xs = [torch.from_numpy(a.view(np.int16)).to(dev).view(torch.bfloat16) for a in imgs]
            gs = [torch.from_numpy(a.view(np.int16)).to(dev).view(torch.bfloat16) for a in grads]
        else:
            xs = [torch.from_numpy(G.bf16_bits_to_f32(a)).to(dev) for a in imgs]
            gs = [torch.from_numpy(G.bf16_bits_to_f32(a)).to(dev) for a in grads]
        ys = [torch.empty_like(v) for v in xs]
        zs = [torch.empty_like(v) for v in gs]
        pf = PL.Plan2D(xs, ys, 4)
        pb = PL.Plan2D(gs, zs, 4, inverse=True)

        def fb():
            pf.execute()
            pb.execute()
        ms5 = _timed(fb, 10, 2, st)
        ms5g = _timed(_graphed(fb, st), 10, 2, st)
        nel = sum(v.numel() for v in xs)
        res[f"ms_{name}"] = round(ms5, 4)
        res[f"gbps_{name}"] = round(4 * nel * xs[0].element_size() / (ms5 * 1e-3) / 1e9, 1)
        res[f"ms_{name}_graph"] = round(ms5g, 4)
        res[f"gbps_{name}_graph"] = round(4 * nel * xs[0].element_size() / (ms5g * 1e-3) / 1e9, 1)
        res[f"elements_per_s_{name}"] = round(2 * nel / (ms5 * 1e-3) / 1e9, 2)
        del xs, gs, ys, zs, pf, pb
        torch.cuda.empty_cache()
    res["unit_elements_per_s"] = "G elements/s, fwd + bwd"
    print(json.dumps(res), flush=True)

    # 4b) the plain 2D kernels on the 4096^2 image, 5 levels, in 16-bit
    #     storage: each kernel's duration under the headline protocol (16
    #     rotating sets, start event queued behind 16 untimed launches)
    from paper_1002_2184_amd import _abi
    x0 = torch.from_numpy(G.config2()).to(dev)
    for name, dt, code in (("bf16", torch.bfloat16, 1), ("f16", torch.float16, 2)):
        xs16 = [x0.to(dt) for _ in range(16)]
        ys16 = [torch.empty_like(v) for v in xs16]
        zs16 = [torch.empty_like(v) for v in xs16]
        q = st.cuda_stream

        def per_launch(fn, reps=400):
            for k in range(128):
                fn(k % 16)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(st)
            for k in range(reps):
                fn(k % 16)
            e1.record(st)
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) / reps
        us_f = 1e3 * per_launch(lambda k: _abi.check(_abi.haar_fwd_2d(
            xs16[k].data_ptr(), ys16[k].data_ptr(), H, W, LEVELS, 1, code, q)))
        us_i = 1e3 * per_launch(lambda k: _abi.check(_abi.haar_inv_2d(
            ys16[k].data_ptr(), zs16[k].data_ptr(), H, W, LEVELS, 1, code, q)))
        nb = 2 * H * W * 2
        print(json.dumps({"workload": f"2d-smooth-4096x4096-L5 {name} kernels", "us_fwd": round(us_f, 2),
                          "us_inv": round(us_i, 2), "gbps_fwd": round(nb / (us_f * 1e-6) / 1e9, 1),
                          "gbps_inv": round(nb / (us_i * 1e-6) / 1e9, 1),
                          "roundtrip_max_err_over_rms": float((zs16[0].float() - xs16[0].float()).abs().max()
                                                              / xs16[0].float().pow(2).mean().sqrt())}),
              flush=True)
        del xs16, ys16, zs16
    del x0
    torch.cuda.empty_cache()

    # 5) fused shrinkage (analysis -> soft threshold -> synthesis in one HBM
    #    pass) on the 4096^2 image, 5 levels, 16 rotating sets; beside the
    #    same pipeline unfused: fwd2d, torch elementwise threshold, inv2d
    x0 = torch.from_numpy(G.config2()).to(dev)
    sets = 16
    xs = [x0.clone() for _ in range(sets)]
    ys = [torch.empty_like(x0) for _ in range(sets)]
    cs = [torch.empty_like(x0) for _ in range(sets)]
    thr = [40.0, 20.0, 10.0, 5.0, 2.5]
    kk = [0]

    def fused():
        k = kk[0] = (kk[0] + 1) % sets
        T.shrink2d(xs[k], 5, thr, "soft", out=ys[k])

    def unfused():
        k = kk[0] = (kk[0] + 1) % sets
        c = T.fwd2d(xs[k], 5, out=cs[k])
        ll = c[:128, :128].clone()
        c.copy_(torch.sign(c) * torch.clamp(c.abs() - thr[0], min=0.0))
        c[:128, :128] = ll
        T.inv2d(c, 5, out=ys[k])
    ms_f = _timed(fused, 96, 16, st)
    ms_u = _timed(unfused, 32, 8, st)
    nb = 2 * x0.numel() * 4
    print(json.dumps({"workload": "2d-smooth-4096x4096-L5 fused soft shrink",
                      "us_fused": round(ms_f * 1e3, 2), "gbps_fused_one_pass": round(nb / (ms_f * 1e-3) / 1e9, 1),
                      "us_unfused_fwd_threshold_inv": round(ms_u * 1e3, 2),
                      "speedup_vs_unfused": round(ms_u / ms_f, 2)}), flush=True)
    del xs, ys, cs, x0
    torch.cuda.empty_cache()

    # 6) the same in 1D: 256 signals of 65536 samples, 12 levels, one chunk pass
    x1 = torch.randn(256, 65536, device=dev)
    x1s = [x1.clone() for _ in range(4)]
    y1s = [torch.empty_like(x1) for _ in range(4)]
    kk[0] = 0

    def fused1():
        k = kk[0] = (kk[0] + 1) % 4
        T.shrink1d(x1s[k], 12, 0.5, "soft", out=y1s[k])

    def plain1():
        k = kk[0] = (kk[0] + 1) % 4
        T.fwd1d(x1s[k], 12, out=y1s[k])
        T.inv1d(y1s[k], 12, out=x1s[(k + 2) % 4])
    ms_f1 = _timed(fused1, 48, 8, st)
    ms_p1 = _timed(plain1, 24, 4, st)
    nb1 = 2 * x1.numel() * 4
    print(json.dumps({"workload": "1d-256x65536-L12 fused soft shrink",
                      "us_fused": round(ms_f1 * 1e3, 2),
                      "gbps_fused_one_pass": round(nb1 / (ms_f1 * 1e-3) / 1e9, 1),
                      "us_plain_fwd_inv": round(ms_p1 * 1e3, 2),
                      "speedup_vs_fwd_inv": round(ms_p1 / ms_f1, 2)}), flush=True)

    # 7) the direct (convolve-then-decimate) bank of Fig. 1 / Fig. 5 beside
    #    the fast bank, same signals (256 x 65536, 12 levels)
    from paper_1002_2184_amd import _abi
    ws = torch.empty(_abi.haar_direct_workspace_size(x1.shape[1], x1.shape[0]), dtype=torch.uint8, device=dev)
    kk[0] = 0

    def dfwd():
        k = kk[0] = (kk[0] + 1) % 4
        T.direct1d(x1s[k], 12, out=y1s[k], workspace=ws)

    def dinv():
        k = kk[0] = (kk[0] + 1) % 4
        T.direct1d(y1s[k], 12, inverse=True, out=x1s[(k + 2) % 4], workspace=ws)

    def ffwd():
        k = kk[0] = (kk[0] + 1) % 4
        T.fwd1d(x1s[k], 12, out=y1s[k])

    def finv():
        k = kk[0] = (kk[0] + 1) % 4
        T.inv1d(y1s[k], 12, out=x1s[(k + 2) % 4])
    res = {"workload": "1d-256x65536-L12 direct vs fast bank"}
    for name, fn in (("direct_fwd", dfwd), ("direct_inv", dinv), ("fast_fwd", ffwd), ("fast_inv", finv)):
        ms = _timed(fn, 16, 4, st)
        res[f"us_{name}"] = round(ms * 1e3, 2)
        res[f"gbps_{name}"] = round(nb1 / (ms * 1e-3) / 1e9, 1)
    res["fast_speedup_fwd"] = round(res["us_direct_fwd"] / res["us_fast_fwd"], 2)
    res["fast_speedup_inv"] = round(res["us_direct_inv"] / res["us_fast_inv"], 2)
    res["note"] = "GB/s = algorithmic bytes (read + write once) / time"
    print(json.dumps(res), flush=True)

    # 8) separable 3D on CT-like volumes
    volumes()


def volumes():
    """Separable 3D on CT-like volumes: 4 x 256^3, 3 levels (one fused pass)
    in FP32 and BF16, and full depth (8 levels, three passes), beside a
    torch copy of the same bytes.  One JSON line per case."""
    import torch

    from paper_1002_2184_amd import transform as T
    from workloads import generators as G

    dev = torch.device("cuda", 0)
    st = torch.cuda.current_stream(dev)
    kk = [0]
    vol = torch.from_numpy(G.to_storage(G.phantom_volume(G.rng_for(8), 256, 256, 256), G.F32)).to(dev)
    gen = torch.Generator(device=dev)
    gen.manual_seed(G.SEED + 8)
    for dt, L in ((torch.float32, 3), (torch.bfloat16, 3), (torch.float32, 8)):
        vs = [(vol + 0.02 * torch.randn((4, 256, 256, 256), device=dev, generator=gen)).to(dt) for _ in range(4)]
        cs = [torch.empty_like(v) for v in vs]
        nb = 2 * vs[0].numel() * vs[0].element_size()
        kk[0] = 0

        def vf():
            k = kk[0] = (kk[0] + 1) % 4
            T.fwd3d(vs[k], L, out=cs[k])

        def vi():
            k = kk[0] = (kk[0] + 1) % 4
            T.inv3d(cs[k], L, out=vs[(k + 2) % 4])

        def vc():
            k = kk[0] = (kk[0] + 1) % 4
            cs[k].copy_(vs[k])
        res = {"workload": f"3d-phantom-4x256^3-L{L} {str(dt).split('.')[-1]}"}
        for name, fn in (("fwd", vf), ("inv", vi), ("torch_copy", vc)):
            ms = _timed(fn, 20, 4, st)
            res[f"us_{name}"] = round(ms * 1e3, 2)
            res[f"gbps_{name}"] = round(nb / (ms * 1e-3) / 1e9, 1)
        print(json.dumps(res), flush=True)
        del vs, cs


def _oracle_rate(x_np, budget_s: float, max_reps: int):
    """Repeated fwd + inv of the image through the FP64 oracle: (GB/s, reps,
    seconds, threads), GB/s counting the algorithmic bytes of the FP32 step."""
    import numpy as np
    import oracle
    xw = x_np.astype(np.float64)
    orc = oracle.default()
    reps, t0 = 0, time.perf_counter()
    while True:
        y = orc.fwd_2d(xw, LEVELS)
        orc.inv_2d(y, LEVELS)
        reps += 1
        el = time.perf_counter() - t0
        if el >= budget_s or reps >= max_reps:
            break
    return 4.0 * H * W * 4 * reps / el / 1e9, reps, el, orc.num_threads()


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(x_np, budget_s: float):
    """The FP64 oracle (fwd + inv of the same image) on all of this host's
    cores, and on one core (a child process with OMP_NUM_THREADS=1)."""
    import subprocess
    gbps, reps, el, thr = _oracle_rate(x_np, budget_s, 20)
    out = {"value": round(gbps, 4), "unit": "GB/s", "cores": thr, "kind": "oracle",
           "sample": f"{reps} x (5-level fwd + inv of the 4096x4096 image), FP64, {el:.1f} s",
           "cpu_model": _cpu_model(), "host_cpus": os.cpu_count()}
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-one-core", str(budget_s)],
                       capture_output=True, text=True, env=env, timeout=300)
    try:
        one = json.loads(r.stdout.strip().splitlines()[-1])
        out["one_core"] = {"value": one["value"], "unit": "GB/s", "cores": one["cores"],
                           "sample": one["sample"]}
    except (ValueError, IndexError, KeyError):
        out["one_core"] = None
    return out


def cpu_one_core(budget_s: float):
    """The one-core leg of the CPU baseline (run with OMP_NUM_THREADS=1)."""
    from workloads import generators as G
    gbps, reps, el, thr = _oracle_rate(G.config2(H, W), budget_s, 4)
    print(json.dumps({"value": round(gbps, 4), "cores": thr,
                      "sample": f"{reps} x (5-level fwd + inv of the 4096x4096 image), FP64, {el:.1f} s"}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--pmc-probe", action="store_true",
                    help="run the dispatches profiled by the rocprofv3 counter passes and exit")
    ap.add_argument("--write-traffic", nargs=3, metavar=("FETCH_CSV", "WRITE_CSV", "COMMAND"),
                    help="summarise two rocprofv3 counter CSVs into the profiles/ traffic file")
    ap.add_argument("--pmc-probe-kind", choices=sorted(PMC_KINDS),
                    help="run the dispatches of one of the other counter probes and exit")
    ap.add_argument("--write-traffic-kind", nargs=5, metavar=("KIND", "FETCH_CSV", "WRITE_CSV", "COMMAND", "OUT_MD"),
                    help="summarise the counter passes of --pmc-probe-kind into a profiles/ Markdown table")
    ap.add_argument("--write-kernel-stats", nargs=3, metavar=("STATS_CSV", "COMMAND", "OUT_MD"),
                    help="summarise a rocprofv3 kernel stats CSV into a Markdown table")
    ap.add_argument("--suite", action="store_true",
                    help="measure the other workloads (1D latency, batched, autograd, BF16) and exit")
    ap.add_argument("--volumes", action="store_true",
                    help="measure only the 3D volume workloads of the suite and exit")
    ap.add_argument("--cpu-one-core", type=float, metavar="BUDGET_S",
                    help="internal: the one-core leg of the CPU baseline")
    args = ap.parse_args()
    if args.cpu_one_core is not None:
        cpu_one_core(args.cpu_one_core)
        return
    if args.suite:
        suite()
        return
    if args.volumes:
        volumes()
        return
    if args.pmc_probe_kind:
        pmc_probe_kind(args.pmc_probe_kind)
        return
    if args.write_traffic_kind:
        write_traffic_kind(*args.write_traffic_kind)
        return
    if args.write_kernel_stats:
        write_kernel_stats(*args.write_kernel_stats)
        return
    if args.write_traffic:
        write_traffic(*args.write_traffic)
        return
    if args.pmc_probe:
        pmc_probe()
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(the transform shards by batch items or row stripes without communication; "
              "see the design notes)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1002_2184_amd import _abi
    from paper_1002_2184_amd import autograd as AG
    from paper_1002_2184_amd import transform as T
    from workloads import generators as G

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    x_np = G.config2(H, W)
    x0 = torch.from_numpy(x_np).to(dev)
    xs = [x0.clone() for _ in range(SETS)]
    ys = [torch.empty_like(x0) for _ in range(SETS)]
    zs = [torch.empty_like(x0) for _ in range(SETS)]
    stream = torch.cuda.current_stream(dev)
    n = H * W
    alg_step = 4.0 * n * 4          # fwd: read + write; inv: read + write (FP32)
    alg_launch = 2.0 * n * 4

    # Steps are independent (each works on its own buffer set), so they are
    # issued round-robin on NSTREAMS streams: the ramp and the tail of one
    # step's kernels overlap another step's, as for any stream of independent
    # transforms.  Within a step the synthesis follows its own analysis on the
    # same stream.  Set s always runs on stream s % NSTREAMS (SETS is a
    # multiple of NSTREAMS), so no buffer is shared between streams.
    streams = [stream] + [torch.cuda.Stream(dev) for _ in range(NSTREAMS - 1)]

    # the steps call the C ABI through its binding with the stream handle
    # (pointers taken once), which keeps the host ahead of the device
    sh = [q.cuda_stream for q in streams]
    xp, yp, zp = ([t.data_ptr() for t in ts] for ts in (xs, ys, zs))

    def step(k, nstreams=NSTREAMS):
        s, q = k % SETS, sh[k % nstreams]
        _abi.check(_abi.haar_fwd_2d(xp[s], yp[s], H, W, LEVELS, 1, 0, q))
        _abi.check(_abi.haar_inv_2d(yp[s], zp[s], H, W, LEVELS, 1, 0, q))

    def timed_steps(nstreams):
        """ms per step of K steps on nstreams streams, bracketed by events on
        the main stream that every other stream joins."""
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0.record(stream)
        for q in streams[1:nstreams]:
            q.wait_stream(stream)
        for k in range(args.steps):
            step(k, nstreams)
        for q in streams[1:nstreams]:
            stream.wait_stream(q)
        t1.record(stream)
        torch.cuda.synchronize()
        return t0.elapsed_time(t1) / args.steps

    for k in range(args.warmup):
        step(k)
    torch.cuda.synchronize()

    # headline: K steps bracketed by events
    ms_step = timed_steps(NSTREAMS)
    gbps = alg_step / (ms_step * 1e-3) / 1e9
    # the same steps one after another on a single stream
    for k in range(args.warmup):
        step(k, 1)
    ms_step_one = timed_steps(1)

    # average duration of each kernel: back-to-back launches of it alone,
    # bracketed by HIP events on the launch stream (the sets still rotate, so
    # every launch reads data last touched 15 launches earlier).  The start
    # event is queued behind 512 untimed launches (about 13 ms of work): the
    # timed ones are already queued when it fires, and the device has left
    # the slower state it runs in for the first several milliseconds of
    # sustained work (the same kernel measured 0.5-0.7 us longer when it was
    # the first thing timed, and still 0.5 us longer after 5 ms of work).
    # The figure is the kernel's steady-state duration.  At
    # least 200 launches, in 10 blocks with an event between blocks: the
    # average over all of them, and the 10th / 50th / 90th percentile of the
    # block averages (us).
    def per_launch_ms(fn):
        blocks = 10
        per = max(args.steps, 200) // blocks
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(blocks + 1)]
        torch.cuda.synchronize()
        for k in range(512):
            fn(k % SETS)
        ev[0].record(stream)
        for b in range(blocks):
            for k in range(per):
                fn((b * per + k) % SETS)
            ev[b + 1].record(stream)
        torch.cuda.synchronize()
        means = sorted(ev[b].elapsed_time(ev[b + 1]) / per * 1e3 for b in range(blocks))
        spread = {"p10": round(means[1], 3), "p50": round(statistics.median(means), 3),
                  "p90": round(means[-2], 3)}
        return ev[0].elapsed_time(ev[-1]) / (blocks * per), spread

    q0 = stream.cuda_stream
    fwd_avg, fwd_spread = per_launch_ms(
        lambda s: _abi.check(_abi.haar_fwd_2d(xp[s], yp[s], H, W, LEVELS, 1, 0, q0)))
    inv_avg, inv_spread = per_launch_ms(
        lambda s: _abi.check(_abi.haar_inv_2d(yp[s], zp[s], H, W, LEVELS, 1, 0, q0)))

    # correctness spot check of the timed outputs (GPU side)
    rt_err = float((zs[0] - xs[0]).abs().max() / xs[0].pow(2).mean().sqrt())

    # autograd fwd + bwd (backward = synthesis on the upstream gradient); the
    # upstream gradients rotate with the inputs so every step reads cold data.
    # Eager steps are bound by the host (autograd bookkeeping, allocation);
    # the graph-captured step measures the device work of the same calls.
    gs = [torch.randn(H, W, device=dev) for _ in range(SETS)]
    xr = [x.clone().requires_grad_(True) for x in xs]

    def ag_step(k):
        s = k % SETS
        y = AG.HaarFwd2D.apply(xr[s], LEVELS)
        (gx,) = torch.autograd.grad(y, xr[s], gs[s])
        return gx

    def timed_loop(fn):
        a0 = torch.cuda.Event(enable_timing=True)
        a1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a0.record(stream)
        for k in range(args.steps):
            fn(k)
        a1.record(stream)
        torch.cuda.synchronize()
        return a0.elapsed_time(a1) / args.steps

    for k in range(args.warmup):
        ag_step(k)
    torch.cuda.synchronize()
    ag_eager_ms = timed_loop(ag_step)

    side = torch.cuda.Stream(dev)
    side.wait_stream(stream)
    with torch.cuda.stream(side):
        for k in range(3):
            ag_step(k)
    stream.wait_stream(side)
    torch.cuda.synchronize()
    # one replay = one step on each buffer set, the steps alternating between
    # the streams as in the headline (forked from and joined to the capture
    # stream inside the capture)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        cap = torch.cuda.current_stream(dev)
        for q in streams[1:]:
            q.wait_stream(cap)
        for s_ in range(SETS):
            with torch.cuda.stream(streams[s_ % NSTREAMS] if s_ % NSTREAMS else cap):
                ag_step(s_)
        for q in streams[1:]:
            cap.wait_stream(q)
    torch.cuda.synchronize()
    graph.replay()
    reps = max(1, args.steps // SETS)
    a0 = torch.cuda.Event(enable_timing=True)
    a1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a0.record(stream)
    for _ in range(reps):
        graph.replay()
    a1.record(stream)
    torch.cuda.synchronize()
    ag_ms = a0.elapsed_time(a1) / (reps * SETS)
    ag_gbps = alg_step / (ag_ms * 1e-3) / 1e9

    dom, dom_ms = ("fwd2d", fwd_avg) if fwd_avg >= inv_avg else ("inv2d", inv_avg)
    achieved = alg_launch / (dom_ms * 1e-3) / 1e9
    traffic = load_traffic(dom)
    out = {
        "metric": METRIC,
        "value": round(gbps, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "2d-smooth-4096x4096-L5 fwd+inv", "height": H, "width": W,
                   "levels": LEVELS, "storage": "f32", "buffer_sets": SETS,
                   "cold_cache": f"{SETS} rotating buffer sets, {(SETS - 1) * 2 * n * 4 >> 20} MiB "
                                 "read between reuses of a set",
                   "streams": NSTREAMS,
                   "schedule": f"independent steps round-robin on {NSTREAMS} streams; each step's synthesis "
                               "follows its own analysis"},
        "one_stream": {"value": round(alg_step / (ms_step_one * 1e-3) / 1e9, 2),
                       "ms_per_step": round(ms_step_one, 5),
                       "pct_of_hbm_peak": round(100.0 * alg_step / (ms_step_one * 1e-3) / 1e9 / PEAK_GBPS, 2)},
        "pct_of_hbm_peak": round(100.0 * gbps / PEAK_GBPS, 2),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": PEAK_GBPS,
                     "unit": "GB/s", "frac": round(achieved / PEAK_GBPS, 4),
                     "traffic": traffic, "kernel": dom,
                     "avg_launch_us": round(dom_ms * 1e3, 3),
                     "bytes_per_launch": int(alg_launch)},
        "kernels_avg_us": {"fwd2d": round(fwd_avg * 1e3, 3), "inv2d": round(inv_avg * 1e3, 3)},
        "kernels_block_us": {"fwd2d": fwd_spread, "inv2d": inv_spread},
        "fwd_bwd": {"value": round(ag_gbps, 2), "unit": "GB/s", "ms_per_step": round(ag_ms, 5),
                    "vs_plain_fwd_inv": round(ag_gbps / gbps, 4),
                    "how": f"HaarFwd2D.apply + torch.autograd.grad on each buffer set, the steps round-robin on "
                           f"{NSTREAMS} streams, captured in one HIP graph",
                    "eager_ms_per_step": round(ag_eager_ms, 5),
                    "eager_value": round(alg_step / (ag_eager_ms * 1e-3) / 1e9, 2)},
        "roundtrip_max_err_over_rms": rt_err,
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(x_np, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
