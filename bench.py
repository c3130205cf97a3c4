"""Benchmark: FP32 FFT-demag + RK4 LLG steps on one MI355X.

Workload ``cube128``: a 128^3 cube of 2 nm cells (padded FFT grid 256^3),
Ms 1e6 A/m, A 1.5e-11 J/m, Ku 5e4 J/m^3 along x, alpha 0.1, gamma0 2.211e5,
dt 1e-14 s, isotropic random initial M (seed 3128); synthetic data.  A step
is one classical RK4 step: four demag evaluations and four field + LLG
stages, all on the GPU with the state resident in HBM.  With the fused
schedule (the default) a step is XFWD(M) once, then per stage YFWD, ZCONV,
YINV and one fused launch (x inverse of the field, the stage, x forward of
the stage's result).  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload cube128]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s


ORDER_NAMES = {0: "default radix order", 1: "radix order 1 (radix 16 first; radix 3 then 4s)",
               2: "radix order 2 (radix 4 only)"}


def describe_tiles(tiles):
    """The launch configuration of every pass in words, from the tile codes
    (P + 256 * variant; the stage kernel's vector width; the fused stage
    pass's P + 256 * log2 W, 0 = the unfused path)."""
    out = {}
    for name, t in tiles.items():
        if not t:
            continue
        P, v = t & 255, t >> 8
        if name == "stage":
            out[name] = "%d cells per thread" % t
        elif name == "xstage":
            out[name] = "fused x inverse + stage + x forward, %d row pairs per workgroup, %d cells per stage task" % (
                P, 1 << v) if t else "unfused (x inverse, stage kernel, x forward)"
        elif name in ("zconv", "yconv"):
            kind = {0: "three components in registers, " + ORDER_NAMES[0],
                    1: "component split, default values per thread", 2: "component split, twice the values per thread",
                    3: "three components in registers, " + ORDER_NAMES[1],
                    4: "three components in registers, " + ORDER_NAMES[2]}.get(v, "variant %d" % v)
            out[name] = "%d columns per workgroup, %s" % (P, kind)
        elif name != "reduce":
            kind = {0: ORDER_NAMES[0], 1: ORDER_NAMES[0] + ", twice the values per thread",
                    2: ORDER_NAMES[1], 3: ORDER_NAMES[2]}.get(v, "variant %d" % v)
            unit = "row pairs" if name in ("xfwd", "xinv") else "columns"
            out[name] = "%d %s per workgroup, %s" % (P, unit, kind)
    return out


def pass_bytes(nx, ny, nz):
    """Algorithmic bytes per launch of each kernel kind (compulsory reads and
    writes of the pruned five-pass schedule; neighbour re-reads not counted)."""
    N = nx * ny * nz
    nc = 3 * nz * ny * (nx + 1)           # X1 complex elements
    nc2 = 3 * nz * 2 * ny * (nx + 1)      # X2 complex elements
    nK = 6 * (nz + 1 if nz > 1 else 1) * (ny + 1) * (nx + 1)
    b = {
        "xfwd": 4 * 3 * N + 8 * nc,
        "xinv": 8 * nc + 4 * 3 * N,
    }
    if nz > 1:
        b["yfwd"] = 8 * nc + 8 * nc2
        b["zconv"] = 8 * nc2 * 2 + 4 * nK
        b["yinv"] = 8 * nc2 + 8 * nc
    else:
        b["yconv"] = 8 * nc * 2 + 4 * (4 * (ny + 1) * (nx + 1))
    # RK4 stages read/write 48N, 72N, 72N, 60N bytes: mean per launch
    b["stage"] = (48 + 72 + 72 + 60) * N / 4.0
    # fused x-inverse / stage / x-forward: the half spectrum in (8 nc), the
    # stage without its field (36N, 60N, 60N, 48N) and the new state's half
    # spectrum out (8 nc; not after stage 4): mean per launch
    b["xstage"] = ((36 + 60 + 60 + 48) * N + (16 + 16 + 16 + 8) * nc) / 4.0
    return b


XSTAGE_BYTES = {1: (36, 16), 2: (60, 16), 3: (60, 16), 4: (48, 8)}  # (x N, x nc) per RK4 stage


def step_bytes(nx, ny, nz, fused=True):
    """Algorithmic bytes of one RK4 step: the unfused schedule runs four
    complete demag evaluations and four stage kernels; the fused one runs
    XFWD once, the middle passes four times and four fused launches."""
    b = pass_bytes(nx, ny, nz)
    mid = sum(v for k, v in b.items() if k in ("yfwd", "zconv", "yinv", "yconv"))
    if not fused:
        return 4 * (b["xfwd"] + mid + b["xinv"] + b["stage"])
    return b["xfwd"] + 4 * mid + 4 * b["xstage"]


# the sources the demag passes and the stage kernel are built from (the
# kernels whose counters the traffic summary holds)
PROFILED_SOURCES = ("fft_engine.hpp", "demag_kernels.hpp", "demag.hip", "layout.hpp", "stage_body.hpp", "llg.hip",
                    "mm_internal.hpp", "xstage_body.hpp", "xstage.hip")


def kernel_source_hash():
    h = hashlib.sha256()
    for f in PROFILED_SOURCES:
        with open(os.path.join(ROOT, "paper_1406_7459_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic(workload, kernel, tile):
    """HBM bytes per launch of pass `kernel` with launch configuration `tile`
    from the committed rocprofv3 counter summary, if it was taken on the
    current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "traffic_%s.txt" % workload)
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_hash") != kernel_source_hash():
        return None
    v = kv.get("hbm_bytes_per_launch.%s.%d" % (kernel, tile))
    return float(v) if v else None


def _workload(name):
    from paper_1406_7459_amd import workloads as W
    return W.cube(int(name[4:])) if name.startswith("cube") else getattr(W, name)()


def pass_tile_of(kname, blocks, threads, shape):
    """(pass, tile, sub) of a dispatch of this library on a grid of `shape`
    from its kernel name, its number of workgroups (every launch of the
    library is one-dimensional) and its total threads: sub is the RK4 stage
    (0 = Euler) for the stage kernel, whose tile is its vector width, and 0
    otherwise; None for anything else (other transform lengths, set-up
    kernels)."""
    import re
    nx, ny, nz = shape
    nxc, pairs = nx + 1, (3 * nz * ny + 1) // 2
    blocks = max(1, blocks)

    def p2(x):
        p = 1
        while p < x:
            p *= 2
        return p

    lens = {"xfwd": 2 * nx, "xinv": 2 * nx, "yfwd": 2 * ny, "yinv": 2 * ny, "yconv": 2 * ny, "zconv": 2 * nz}

    def col_P(nrows, edge):
        # the column passes' workgroup count for P: tiles over the nx columns
        # below the last plus edge workgroups for the last when P divides nx
        # (and edge launches are used), else tiles over all nx + 1 columns
        for P in (1, 2, 4, 8, 16, 32, 64, 128):
            if edge and P > 1 and nx % P == 0:
                n = nx // P * nrows + -(-nrows // P)
            else:
                n = -(-nxc // P) * nrows
            if n == blocks:
                return P
        return p2(-(-nxc * nrows // blocks))

    m = re.search(r"mmk::k_(xfwd|yfwd|yinv|xinv)<(\d+), (\d+)>", kname)
    if m:
        if int(m.group(2)) != lens[m.group(1)]:
            return None
        rows = m.group(1) in ("xfwd", "xinv")
        P = p2(-(-pairs // blocks)) if rows else col_P(3 * nz, True)
        return m.group(1), P + 256 * int(m.group(3)), 0
    m = re.search(r"mmk::k_conv_reg3<(\d+), (true|false), (\d)>", kname)
    if m:
        z = m.group(2) == "true"
        pname = "zconv" if z else "yconv"
        order = int(m.group(3))
        var = 0 if order == 0 else 2 + order
        P = col_P(2 * ny, True) if z else col_P(1, False)
        return (pname, P + 256 * var, 0) if int(m.group(1)) == lens[pname] else None
    m = re.search(r"mmk::k_conv_split<(\d+), (\d+), (true|false)>", kname)
    if m:
        z = m.group(3) == "true"
        pname = "zconv" if z else "yconv"
        if int(m.group(1)) != lens[pname]:
            return None
        return pname, col_P(2 * ny if z else 1, False) + 256 * (1 + int(m.group(2))), 0
    m = re.search(r"mmk::k_xstage<(\d+), ([0-4]), (true|false), (\d)>", kname)
    if m:
        if int(m.group(1)) != lens["xfwd"]:
            return None
        w = {1: 0, 2: 1, 4: 2}[int(m.group(4))]
        return "xstage", p2(-(-(nz * ny) // (2 * blocks))) + 256 * w, int(m.group(2))
    m = re.search(r"mmk::k_stage(_vec)?<([0-4])(?:, (\d))?>", kname)
    w = int(m.group(3)) if m and m.group(3) else 1
    if m and threads * w >= nx * ny * nz:
        return "stage", w, int(m.group(2))
    return None


def summarize_trace(workload, db):
    """Text of profiles/kernels_<workload>.txt from a rocprofv3 --kernel-trace
    database of bench.py: per (pass, tile) of the workload's grid, the
    dispatch count and durations (the autotuner's candidates appear as their
    own rows), then the other kernels by name."""
    import sqlite3
    import statistics
    shape = _workload(workload).shape
    con = sqlite3.connect(db)
    groups, other = {}, {}
    for name, gx, gy, gz, wx, wy, wz, dur in con.execute(
            "select name, grid_x, grid_y, grid_z, workgroup_x, workgroup_y, workgroup_z, duration from kernels"):
        key = pass_tile_of(name, gx // max(1, wx), gx * gy * gz, shape)
        if key:
            groups.setdefault(key, []).append(dur / 1e3)
        else:
            other.setdefault(name.split("(")[0].replace("void ", ""), []).append(dur / 1e3)
    alg = pass_bytes(*shape)
    out = ["# kernel trace, %s (%dx%dx%d cells), rocprofv3 --kernel-trace" % ((workload,) + tuple(shape)),
           "# commands (from /tmp on the GPU, REPO = repository root, OUT = an output folder; the first, a",
           "# full bench run, tunes and writes the tune cache, so the traced run launches the tuned tiles",
           "# without re-tuning):",
           "#   MM_TUNE_CACHE=$OUT/tune.json python3 $REPO/bench.py --workload %s --no-cpu-baseline "
           "--no-batch --no-surrogate" % workload,
           "#   MM_TUNE_CACHE=$OUT/tune.json rocprofv3 --kernel-trace --stats -d $OUT/prof_%s -o %s -- python3 "
           "$REPO/bench.py --workload %s --steps 10 --warmup 2 --no-cpu-baseline --no-batch --no-other-configs "
           "--no-surrogate" % (workload, workload, workload),
           "#   python3 bench.py --summarize-trace %s $OUT/prof_%s/%s_results.db" % (workload, workload, workload),
           "# durations in microseconds; tile = P + 256 * variant, for the stage kernel its vector width, for",
           "# the fused xstage pass its row pairs per workgroup, with the RK4 stage (1-4, 0 = Euler) in column s;",
           "# GB/s from the algorithmic bytes per launch (bench.pass_bytes; stage: 48N, 72N, 72N, 60N bytes,",
           "# Euler 60N; xstage: 36N, 60N, 60N, 48N plus 16, 16, 16, 8 bytes per half-spectrum element)",
           "# over the median duration",
           "%-7s %6s %2s %6s %9s %9s %9s %9s %8s" % ("pass", "tile", "s", "calls", "median", "mean", "min", "max", "GB/s")]
    N = shape[0] * shape[1] * shape[2]
    nc = 3 * shape[2] * shape[1] * (shape[0] + 1)
    stage_bytes = {0: 60 * N, 1: 48 * N, 2: 72 * N, 3: 72 * N, 4: 60 * N}
    xs_bytes = {k: a * N + b * nc for k, (a, b) in XSTAGE_BYTES.items()}
    for key in sorted(groups):
        pname, tile, sub = key
        d = groups[key]
        med = statistics.median(d)
        a = stage_bytes[sub] if pname == "stage" else (xs_bytes.get(sub) if pname == "xstage" else alg.get(pname))
        out.append("%-7s %6d %2d %6d %9.2f %9.2f %9.2f %9.2f %8s" % (
            pname, tile, sub, len(d), med, statistics.mean(d), min(d), max(d), ("%.0f" % (a / med / 1e3)) if a else "-"))
    out.append("# other kernels")
    for name in sorted(other, key=lambda n: -sum(other[n])):
        d = other[name]
        out.append("#   %-56s calls %6d mean %9.2f total %10.1f" % (name[:56], len(d), statistics.mean(d), sum(d)))
    return "\n".join(out) + "\n"


SQ_SETS = {
    "sq_A": ("SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_LDS", "SQ_INSTS_SALU", "SQ_INSTS_VMEM_RD", "SQ_INSTS_VMEM_WR",
             "SQ_WAVE_CYCLES", "SQ_BUSY_CYCLES"),
    "sq_B": ("SQ_ACTIVE_INST_VALU", "SQ_ACTIVE_INST_LDS", "SQ_LDS_BANK_CONFLICT", "SQ_WAIT_INST_ANY", "SQ_WAIT_ANY",
             "SQ_ACTIVE_INST_ANY", "SQ_WAVE_CYCLES", "SQ_WAVES"),
}


def summarize_counters(workload, pmc_dir, trace_db):
    """Text of profiles/sq_<workload>.txt from the rocprofv3 --pmc databases
    sq_A and sq_B under pmc_dir (the counter sets of SQ_SETS, one run each)
    and a --kernel-trace database of the same tiles for durations: per (pass,
    tile, stage) the median per dispatch of each counter, summed over the
    chip, and ratios of counters in the same units."""
    import glob
    import sqlite3
    import statistics
    shape = _workload(workload).shape
    vals = {}
    for kind, names in SQ_SETS.items():
        db = glob.glob(os.path.join(pmc_dir, kind, "*.db"))[0]
        con = sqlite3.connect(db)
        per = {}
        for disp, kname, gx, wx, gt, cname, v in con.execute(
                "select dispatch_id, kernel_name, grid_size_x, workgroup_size_x, grid_size, counter_name, value "
                "from counters_collection"):
            key = pass_tile_of(kname, gx // max(1, wx), gt, shape)
            if key is None:
                continue
            e = per.setdefault(disp, (key, {}))
            e[1][cname] = e[1].get(cname, 0.0) + v
        for key, cv in per.values():
            for c, v in cv.items():
                vals.setdefault(key, {}).setdefault(c, []).append(v)
    dur = {}
    con = sqlite3.connect(trace_db)
    for name, gx, gy, gz, wx, d in con.execute(
            "select name, grid_x, grid_y, grid_z, workgroup_x, duration from kernels"):
        key = pass_tile_of(name, gx // max(1, wx), gx * gy * gz, shape)
        if key:
            dur.setdefault(key, []).append(d / 1e3)
    out = ["# SQ counters per launch, %s (%dx%dx%d cells), rocprofv3 --pmc" % ((workload,) + tuple(shape)),
           "# commands (from /tmp on the GPU, REPO = repository root, OUT = an output folder; the tune cache",
           "# written by a full bench run, so these runs launch the tuned tiles without re-tuning):",
           "#   MM_TUNE_CACHE=$OUT/tune.json python3 $REPO/bench.py --workload %s --no-cpu-baseline --no-batch "
           "--no-surrogate" % workload]
    for kind, names in SQ_SETS.items():
        out.append("#   MM_TUNE_CACHE=$OUT/tune.json rocprofv3 --pmc %s -d $OUT/sq/%s -o %s -- python3 $REPO/bench.py "
                   "--workload %s --steps 3 --warmup 1 --no-cpu-baseline --no-batch --no-other-configs "
                   "--no-surrogate" % (" ".join(names), kind, kind, workload))
    out += ["#   python3 bench.py --summarize-counters %s $OUT/sq $OUT/prof_%s/%s_results.db"
            % (workload, workload, workload),
            "# columns: waves; VALU, LDS, SALU, VMEM instructions per wave; valu_floor_us = SQ_INSTS_VALU x 4",
            "# cycles (a wave64 FP32 VALU op without packed math) / (1024 SIMDs x 2.4 GHz); the trace median",
            "# duration; valu_frac = floor / median; lds_conf = SQ_LDS_BANK_CONFLICT / SQ_ACTIVE_INST_LDS;",
            "# wait = SQ_WAIT_INST_ANY / SQ_WAVE_CYCLES (share of wave time waiting on a dependency);",
            "# w_any = SQ_WAIT_ANY / SQ_WAVE_CYCLES (waiting on anything, barriers included);",
            "# valu_act = SQ_ACTIVE_INST_VALU / SQ_WAVE_CYCLES",
            "%-7s %5s %2s %7s %6s %6s %5s %6s %7s %8s %7s %6s %6s %6s %6s %6s" % (
                "pass", "tile", "s", "waves", "valu", "lds", "salu", "vmem", "floor", "median", "v_frac",
                "ldsc", "wait", "w_any", "v_act", "n")]
    for key in sorted(vals):
        c = {k: statistics.median(v) for k, v in vals[key].items()}
        w = c.get("SQ_WAVES", 0.0)
        if not w:
            continue
        floor = c.get("SQ_INSTS_VALU", 0.0) * 4 / (1024 * 2.4e3)
        med = statistics.median(dur[key]) if key in dur else float("nan")
        wc = c.get("SQ_WAVE_CYCLES", 0.0) or float("nan")
        lds_act = c.get("SQ_ACTIVE_INST_LDS", 0.0) or float("nan")
        out.append("%-7s %5d %2d %7d %6.0f %6.0f %5.0f %6.1f %7.2f %8.2f %7.2f %6.3f %6.3f %6.3f %6.3f %6d" % (
            key[0], key[1], key[2], w, c.get("SQ_INSTS_VALU", 0) / w, c.get("SQ_INSTS_LDS", 0) / w,
            c.get("SQ_INSTS_SALU", 0) / w, (c.get("SQ_INSTS_VMEM_RD", 0) + c.get("SQ_INSTS_VMEM_WR", 0)) / w,
            floor, med, floor / med, c.get("SQ_LDS_BANK_CONFLICT", 0) / lds_act,
            c.get("SQ_WAIT_INST_ANY", 0) / wc, c.get("SQ_WAIT_ANY", 0) / wc, c.get("SQ_ACTIVE_INST_VALU", 0) / wc,
            len(vals[key].get("SQ_WAVES", []))))
    return "\n".join(out) + "\n"


def summarize_traffic(workload, pmc_dir):
    """Text of profiles/traffic_<workload>.txt from four rocprofv3 --pmc
    databases under pmc_dir: sweep_FETCH_SIZE, sweep_WRITE_SIZE (bench.py
    --sweep-tiles) and copy_FETCH_SIZE, copy_WRITE_SIZE (--calibrate-copy).
    Each counter is scaled by what it reads for the 512 MiB copy; per pass
    and tile the median over that configuration's dispatches is kept."""
    import glob
    import sqlite3
    import statistics

    def load(kind, counter):
        db = glob.glob(os.path.join(pmc_dir, "%s_%s" % (kind, counter), "*.db"))[0]
        con = sqlite3.connect(db)
        per = {}
        for disp, kname, gx, wx, gt, v in con.execute(
                "select dispatch_id, kernel_name, grid_size_x, workgroup_size_x, grid_size, value "
                "from counters_collection where counter_name = ?", (counter,)):
            e = per.setdefault(disp, [kname, gx // max(1, wx), gt, 0.0])
            e[3] += v
        return per

    copy_bytes = 512 * 1024 * 1024
    scale = {}
    for c in ("FETCH_SIZE", "WRITE_SIZE"):
        vals = [e[3] for e in load("copy", c).values() if "MulFunctor" in e[0]]
        scale[c] = copy_bytes / (1024.0 * statistics.median(vals))
    shape = _workload(workload).shape
    nx, ny, nz = shape
    acc = {}
    for c in ("FETCH_SIZE", "WRITE_SIZE"):
        for kname, gx, wx, v in load("sweep", c).values():
            key = pass_tile_of(kname, gx, wx, shape)
            if key and not (key[0] in ("stage", "xstage") and key[2] == 0):
                acc.setdefault(key, {}).setdefault(c, []).append(v * 1024.0 * scale[c])
    alg = pass_bytes(nx, ny, nz)
    out = ["# HBM traffic per launch, %s (%dx%dx%d cells), rocprofv3 hardware counters" % (workload, nx, ny, nz),
           "# commands (from /tmp on the GPU, REPO = repository root, OUT = an output folder):",
           "#   rocprofv3 --pmc FETCH_SIZE -d $OUT/pmc/sweep_FETCH_SIZE -o sweep -- python3 $REPO/bench.py --sweep-tiles",
           "#   rocprofv3 --pmc WRITE_SIZE -d $OUT/pmc/sweep_WRITE_SIZE -o sweep -- python3 $REPO/bench.py --sweep-tiles",
           "#   rocprofv3 --pmc FETCH_SIZE -d $OUT/pmc/copy_FETCH_SIZE -o copy -- python3 $REPO/bench.py --calibrate-copy",
           "#   rocprofv3 --pmc WRITE_SIZE -d $OUT/pmc/copy_WRITE_SIZE -o copy -- python3 $REPO/bench.py --calibrate-copy",
           "#   python3 bench.py --summarize-traffic %s $OUT/pmc" % workload,
           "# scale: a 512 MiB copy (512 MiB read + 512 MiB written) reads back FETCH_SIZE x%.4f, WRITE_SIZE x%.4f"
           % (scale["FETCH_SIZE"], scale["WRITE_SIZE"]),
           "# per pass and tile (P + 256 * variant): median fetch / write bytes per launch; stage: mean of RK4 stages 1-4",
           "kernel_source_hash: %s" % kernel_source_hash()]
    stage = {}
    for key in sorted(acc):
        pname, tile, sub = key
        d = acc[key]
        if "FETCH_SIZE" not in d or "WRITE_SIZE" not in d:
            continue
        f, w = statistics.median(d["FETCH_SIZE"]), statistics.median(d["WRITE_SIZE"])
        if pname in ("stage", "xstage"):
            stage.setdefault((pname, tile), []).append(f + w)
            continue
        a = alg.get(pname)
        out.append("# %-6s tile %4d: fetch %11.0f write %11.0f  (x%.2f of algorithmic %d)"
                   % (pname, tile, f, w, (f + w) / a if a else 0.0, a or 0))
        out.append("hbm_bytes_per_launch.%s.%d: %.0f" % (pname, tile, f + w))
    for pname, tile in sorted(stage):
        v = sum(stage[(pname, tile)]) / len(stage[(pname, tile)])
        out.append("# %-6s tile %4d: RK4 stages 1-4 mean %.0f (x%.2f of algorithmic %d)"
                   % (pname, tile, v, v / alg[pname], alg[pname]))
        out.append("hbm_bytes_per_launch.%s.%d: %.0f" % (pname, tile, v))
    return "\n".join(out) + "\n"


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline():
    """The CPU oracle (single-threaded FP64 C) timed on the host: one RK4 step
    of the cube workload's material on a 64^3 cube (its own set-up excluded,
    timed separately), and the 128^3 headline grid extrapolated from it by
    the FFT route's N log N cost (labelled as extrapolated)."""
    import math
    import oracle
    from paper_1406_7459_amd import workloads as W
    wl = W.cube(64)
    nx, ny, nz = wl.shape
    t0 = time.perf_counter()
    dm = oracle.Demag(nx, ny, nz, *wl.cell)
    setup = time.perf_counter() - t0
    m = wl.mat
    p = oracle.Params(Ms=m.Ms, A=m.A, Ku=m.Ku, axis=m.axis, alpha=m.alpha, gamma0=m.gamma0,
                      Hext=m.Hext, dt=m.dt)
    M = m.Ms * wl.initial_unit()
    t0 = time.perf_counter()
    M, _ = dm.run(p, M, 1)
    step = time.perf_counter() - t0
    rate = wl.cells / step
    n64, n128 = 8 * 64 ** 3, 8 * 128 ** 3  # padded FFT points
    step128 = step * (n128 * math.log2(n128)) / (n64 * math.log2(n64))
    return dict(value=rate, unit="cell-updates/s", cores=1, kind="oracle",
                host_cpus=os.cpu_count(), cpu_model=cpu_model(),
                sample="cube64 (64^3 cells, the cube workload's material, 2 nm cells): 1 RK4 step "
                       "(4 demag evaluations by the padded FFT route) in %.1f s, oracle set-up "
                       "(Newell tensor and its transform) %.1f s excluded" % (step, setup),
                cube128_extrapolated={"s_per_step": step128, "cell_updates_per_s": 128 ** 3 / step128,
                                      "how": "extrapolated from the cube64 step by N log N of the "
                                             "padded FFT grid (not run)"})


def oracle_error_sample(plan, wl, torch):
    """Relative L2 of the GPU demag field against the oracle's direct sum at
    sampled cells, for a field of 32 random sources at the full grid size."""
    import numpy as np
    import oracle
    from paper_1406_7459_amd import workloads as W
    nx, ny, nz = wl.shape
    M = wl.mat.Ms * W.sparse_sources(nx, ny, nz, 32, seed=77)
    src = np.flatnonzero(np.abs(M).sum(axis=0).ravel())
    obs = np.unique(np.concatenate([src, W.sample_cells(nx * ny * nz, 96, seed=78)]))
    Hg = plan.demag(torch.from_numpy(M.astype(np.float32)).cuda())
    torch.cuda.synchronize()
    Hg = Hg.cpu().numpy().reshape(3, -1)[:, obs].astype(np.float64)
    Ho = oracle.demag_direct_at(M, wl.cell, obs)
    return float(np.linalg.norm(Hg - Ho) / np.linalg.norm(Ho)), int(obs.size)


def batch_measure(torch, mm, W, steps=10, warmup=2):
    """Field-sweep batch (64 films of uneven sizes): batched step against a
    loop over per-instance plans (plain FP32 RK4), same GPU, same states."""
    wls = W.sweep64()
    shapes = [w.shape for w in wls]
    cells = sum(w.cells for w in wls)
    params = [mm.LLGParams.make(Ms=w.mat.Ms, A=w.mat.A, alpha=w.mat.alpha, Hext=w.mat.Hext,
                                dt=w.mat.dt) for w in wls]
    M0 = [torch.from_numpy((w.mat.Ms * w.initial_unit()).astype("float32")).cuda() for w in wls]
    b = mm.Batch(shapes, [w.cell for w in wls])
    b.autotune(reps=3)
    modes = {}
    for mode in ("grouped", "merged"):
        b.set_mode(mode)
        Mm = [m.clone() for m in M0]
        b.step(params, Mm, warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.step(params, Mm, steps)
        torch.cuda.synchronize()
        modes[mode] = dict(ms_per_step=(time.perf_counter() - t0) / steps * 1e3, query=b.query(), M=Mm)
    tb = modes["merged"]["ms_per_step"] * 1e-3
    Mb = modes["merged"]["M"]
    q = modes["merged"]["query"]
    b.close()
    plans = [mm.Plan(*w.shape, *w.cell) for w in wls]
    for p in plans:
        p.autotune(reps=2)
    Ml = [m.clone() for m in M0]
    for p, pa, m in zip(plans, params, Ml):
        p.step(pa, m, warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for p, pa, m in zip(plans, params, Ml):
        p.step(pa, m, steps)
    torch.cuda.synchronize()
    tl = (time.perf_counter() - t0) / steps
    same = all(bool(torch.equal(a, c)) for a, c in zip(Mb, Ml))
    diff = max(float((a - c).norm() / c.norm()) for a, c in zip(Mb, Ml))
    for p in plans:
        p.close()
    return {"workload": "sweep64 (64 films, nx,ny in {64..512}, nz in {1,2,4,8}, seed 4)",
            "cells": cells, "mode": "merged (one launch per pass kind)",
            "launch_kinds": q["groups"], "launches_per_step": q["launches_per_step"],
            "grouped_mode": {"ms_per_step": modes["grouped"]["ms_per_step"],
                             "groups": modes["grouped"]["query"]["groups"],
                             "launches_per_step": modes["grouped"]["query"]["launches_per_step"]},
            "batched_ms_per_step": tb * 1e3, "looped_ms_per_step": tl * 1e3,
            "speedup_vs_looped_plain_fp32": tl / tb,
            "batched_cell_updates_per_s": cells / tb,
            "bitwise_equal_to_looped": same, "max_state_rel_l2_vs_looped": diff,
            "note": "the merged launches run radix order 1 for 3*2^a lengths; the looped plans' "
                    "autotuner picks its own orders, which round differently"}


def surrogate_measure(torch, mm, W, train_s=20.0, steps=20):
    """Learned form on the 256x256x4 film: a short online training on the
    solver's own pairs (train_s seconds), then `steps` gated RK4 steps
    (tolerance 1e-3, exact demag judging every accepted state) against the
    same steps on the plain FP32 path, from the same held-out state; plus the
    time of one network evaluation (6.07e10 FLOP, BF16 matrix cores)."""
    import numpy as np
    from paper_1406_7459_amd.surrogate_train import init_params
    wl = W.film256(0)
    nx, ny, nz = wl.shape
    m = wl.mat
    plan = mm.Plan(nx, ny, nz, *wl.cell)
    plan.autotune(reps=3)
    sur = mm.Surrogate(nx, ny, nz)
    sur.set_params(init_params(6, 5000))
    dm = torch.empty((3, nz, ny, nx), device="cuda")
    dh = torch.empty_like(dm)
    t0 = time.perf_counter()
    pairs, traj, losses = 0, 0, []
    while time.perf_counter() - t0 < train_s:
        w = W.film256(traj)
        p = mm.LLGParams.make(Ms=w.mat.Ms, A=w.mat.A, alpha=w.mat.alpha, gamma0=w.mat.gamma0, Hext=w.mat.Hext,
                              dt=w.mat.dt)
        M = torch.from_numpy((w.mat.Ms * w.initial_unit()).astype("float32")).cuda()
        plan.step(p, M, 20)
        for _ in range(100):
            mm.Surrogate.make_pair(plan, p, M, 1, dm, dh)
            frac = (time.perf_counter() - t0) / train_s
            losses.append(sur.train_step(dm, dh, 3e-4 * 0.1 ** min(1.0, frac)))
            pairs += 1
            if time.perf_counter() - t0 >= train_s:
                break
        traj += 1
    w = W.film256(900)
    p = mm.LLGParams.make(Ms=w.mat.Ms, A=w.mat.A, alpha=w.mat.alpha, gamma0=w.mat.gamma0, Hext=w.mat.Hext,
                          dt=w.mat.dt)
    M0 = torch.from_numpy((w.mat.Ms * w.initial_unit()).astype("float32")).cuda()
    plan.step(p, M0, 20)
    # each driver: one warm-up call, then the best per-step time of five runs
    # of `steps` steps from M0 in one buffer (the exact path's step graph is
    # keyed by the state's address)
    Mx = M0.clone()

    def best_of(run, reps=5):
        best, r = float("inf"), None
        for _ in range(reps):
            Mx.copy_(M0)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            r = run()
            torch.cuda.synchronize()
            best = min(best, (time.perf_counter() - t1) / steps)
        return best, r

    plan.step(p, Mx, 2)
    te, _ = best_of(lambda: plan.step(p, Mx, steps))
    Me = Mx.clone()
    sur.step(plan, p, Mx, 2, tol=1e-3)
    ts, st = best_of(lambda: sur.step(plan, p, Mx, steps, tol=1e-3))
    err = float((Mx - Me).norm() / Me.norm())
    # the same steps with the residuals read back once per 10 steps
    pg = mm.LLGParams.make(Ms=w.mat.Ms, A=w.mat.A, alpha=w.mat.alpha, gamma0=w.mat.gamma0, Hext=w.mat.Hext,
                           dt=w.mat.dt, sur_check_every=10)
    tg, stg = best_of(lambda: sur.step(plan, pg, Mx, steps, tol=1e-3))
    errg = float((Mx - Me).norm() / Me.norm())
    x = torch.randn((3, nz, ny, nx), device="cuda")
    y = torch.empty_like(x)
    # device time of one network evaluation (input normalisation included):
    # events around 200 back-to-back evaluations on the current stream
    for _ in range(30):
        sur.forward(x, y, normalize=True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(200):
        sur.forward(x, y, normalize=True)
    e1.record()
    torch.cuda.synchronize()
    inf = e0.elapsed_time(e1) / 200 * 1e-3
    sur.close()
    plan.close()
    return {"workload": "film256 (256x256x4, 4 nm, alpha 0.1, in-plane |mu0 H| <= 50 mT); pairs from the solver",
            "training": {"seconds": train_s, "pairs": pairs, "pairs_per_s": pairs / train_s,
                         "loss_first": float(np.mean(losses[:20])),
                         "loss_last": float(np.mean(losses[-20:]))},
            "gated_steps": steps, "tol": 1e-3, "stats": st,
            "exact_ms_per_step": te * 1e3, "surrogate_ms_per_step": ts * 1e3,
            "speedup_vs_plain_fp32": te / ts, "state_rel_l2_vs_exact": err,
            "check_every_10": {"stats": stg, "surrogate_ms_per_step": tg * 1e3, "speedup_vs_plain_fp32": te / tg,
                               "state_rel_l2_vs_exact": errg},
            # a gated step is 4 network evaluations (3 stages and the gate's check)
            # plus the rest (stages, the gate's exact demag, copies); the
            # network time per evaluation at which it would equal the exact
            # step (negative: the rest alone exceeds it)
            "rest_ms_per_step": (tg - 4 * inf) * 1e3,
            "breakeven_inference_ms": (te - (tg - 4 * inf)) / 4 * 1e3,
            "inference_ms": inf * 1e3, "inference_tflops": 6.07e10 / inf / 1e12,
            "inference_mfma_frac": 6.07e10 / inf / 2.5e15}


SURROGATE_PROFILE_CMD = (
    "#   rocprofv3 --kernel-trace --stats -d $OUT/prof_sur -o sur -- python3 $REPO/bench.py "
    "--surrogate-profile",
    "#   python3 bench.py --summarize-surrogate $OUT/prof_sur/sur_results.db")


def surrogate_profile(torch, mm):
    """The launches profiles/surrogate_film256.txt is taken from: 20 network
    evaluations (inference) and 10 training steps on the 256x256x4 film."""
    from paper_1406_7459_amd.surrogate_train import init_params
    nx, ny, nz = 256, 256, 4
    sur = mm.Surrogate(nx, ny, nz)
    sur.set_params(init_params(6, 5000))
    x = torch.randn((3, nz, ny, nx), device="cuda")
    y = torch.empty_like(x)
    for _ in range(20):
        sur.forward(x, y, normalize=True)
    dm, dh = x * 1e-3, torch.randn_like(x) * 1e-4
    for _ in range(10):
        sur.train_step(dm, dh, 1e-5)
    torch.cuda.synchronize()
    sur.close()


def _demangle_mmk(name):
    """mmk::name<int/bool template arguments> from an Itanium-mangled kernel
    name of the library's namespace that the trace left mangled (the bf16
    parameter type stops some demanglers); other names pass unchanged."""
    import re
    m = re.match(r"_ZN3mmk(\d+)", name)
    if not m:
        return name
    n = int(m.group(1))
    base, rest = name[m.end():m.end() + n], name[m.end() + n:]
    args = []
    if rest.startswith("I"):
        for kind, val in re.findall(r"L([ib])(\d+)E", rest[1:rest.find("EE") + 1]):
            args.append(val if kind == "i" else ("true" if val == "1" else "false"))
    return "mmk::" + base + ("<%s>" % ", ".join(args) if args else "")


def summarize_surrogate(db):
    """Text of profiles/surrogate_film256.txt from a rocprofv3 --kernel-trace
    database of bench.py --surrogate-profile: per kernel, the dispatch count
    and durations; for the convolutions the rate of the 32 x 32-channel
    3x3x3 product they compute (2*27*32*32 flop per cell, the last layer's 16
    computed output rows: half of that; the packed first layer 2*28*8*32)."""
    import re
    import sqlite3
    import statistics
    N = 256 * 256 * 4
    con = sqlite3.connect(db)
    groups = {}
    for name, dur in con.execute("select name, duration from kernels"):
        k = re.sub(r"\(.*", "", _demangle_mmk(name)).replace("void ", "")
        groups.setdefault(k, []).append(dur / 1e3)
    tot = sum(sum(v) for v in groups.values())
    out = ["# kernel trace of the learned form, film256 (256x256x4 cells), rocprofv3 --kernel-trace",
           "# command (from /tmp on the GPU, REPO = repository root, OUT = an output folder):", *SURROGATE_PROFILE_CMD,
           "# 20 network evaluations, then 10 training steps; durations in microseconds",
           "# k_conv<E, lo, hi>: E = 3 inference hidden layer, 1 last layer, 0 training forward, 2 input",
           "# gradient (GELU derivative fused); TFLOP/s of the computed 32x32-channel product (BF16 peak 2500);",
           "# k_conv_in<E>: the first layer, 4 taps x 8 channels per K step (28 x 8 x 32 computed per cell)",
           "%-44s %6s %9s %9s %7s %8s" % ("kernel", "calls", "median", "mean", "share", "TFLOP/s")]
    for k in sorted(groups, key=lambda k: -sum(groups[k])):
        v = groups[k]
        med = statistics.median(v)
        rate = ""
        m = re.match(r"mmk::k_conv<(\d)", k)
        if k.startswith("mmk::k_conv_in<"):
            # packed first layer: 7 K steps of 4 taps x 8 channels, 32 outputs
            rate = "%.0f" % (2 * 28 * 8 * 32 * N / (med * 1e-6) / 1e12)
        elif m:
            fl = 2 * 27 * 32 * 32 * N * (0.5 if m.group(1) == "1" else 1.0)
            rate = "%.0f" % (fl / (med * 1e-6) / 1e12)
        elif k.startswith("mmk::k_conv_dw"):
            rate = "%.0f" % (2 * 27 * 32 * 32 * N / (med * 1e-6) / 1e12)
        out.append("%-44s %6d %9.2f %9.2f %6.1f%% %8s" % (k[:44], len(v), med, statistics.mean(v),
                                                       100 * sum(v) / tot, rate))
    return "\n".join(out) + "\n"


SUR_SQ_SETS = {
    "sq_A": ("SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_MFMA", "SQ_INSTS_LDS", "SQ_INSTS_VMEM_RD", "SQ_WAVE_CYCLES",
             "SQ_BUSY_CYCLES", "SQ_VALU_MFMA_BUSY_CYCLES"),
    "sq_B": SQ_SETS["sq_B"],
}


def summarize_surrogate_counters(pmc_dir):
    """Text of profiles/sq_surrogate_film256.txt from the two rocprofv3 --pmc
    runs (SUR_SQ_SETS) of bench.py --surrogate-profile under pmc_dir: per
    convolution kernel the median per dispatch of each counter (summed over
    the chip), per-wave instruction counts, the matrix cores' busy time per
    SIMD, and ratios of counters in the same units."""
    import glob
    import re
    import sqlite3
    import statistics
    per = {}
    for kind in SUR_SQ_SETS:
        db = glob.glob(os.path.join(pmc_dir, kind, "**", "*.db"), recursive=True)[0]
        con = sqlite3.connect(db)
        rows = {}
        for disp, kname, cname, v in con.execute(
                "select dispatch_id, kernel_name, counter_name, value from counters_collection"):
            c = rows.setdefault((disp, kname), {})
            c[cname] = c.get(cname, 0.0) + v
        for (disp, kname), cs in rows.items():
            k = re.sub(r"\(.*", "", _demangle_mmk(kname)).replace("void ", "")
            for c, v in cs.items():
                per.setdefault(k, {}).setdefault(c, []).append(v)
    cmd = ["#   rocprofv3 --pmc %s -d $OUT/sq_sur/%s -o %s -- python3 $REPO/bench.py --surrogate-profile"
           % (" ".join(cs), kind, kind) for kind, cs in SUR_SQ_SETS.items()]
    out = ["# SQ counters per launch of the learned form's convolutions, film256 (256x256x4 cells), rocprofv3 --pmc",
           "# commands (from /tmp on the GPU, REPO = repository root, OUT = an output folder):", *cmd,
           "#   python3 bench.py --summarize-surrogate-counters $OUT/sq_sur",
           "# columns: waves; VALU, MFMA, LDS, VMEM-read instructions per wave; mfma_us = SQ_VALU_MFMA_BUSY_CYCLES",
           "# / (1024 SIMDs x 2.4 GHz), the matrix cores' busy time per SIMD (a launch's duration is in",
           "# surrogate_film256.txt); lds_conf = SQ_LDS_BANK_CONFLICT / SQ_ACTIVE_INST_LDS; wait =",
           "# SQ_WAIT_INST_ANY / SQ_WAVE_CYCLES; w_any = SQ_WAIT_ANY / SQ_WAVE_CYCLES; act =",
           "# SQ_ACTIVE_INST_ANY / SQ_WAVE_CYCLES",
           "%-30s %6s %6s %5s %5s %6s %8s %8s %6s %6s %6s" % ("kernel", "waves", "valu", "mfma", "lds", "vmem", "mfma_us",
                                                          "lds_conf", "wait", "w_any", "act")]
    for k in sorted(per):
        if not k.startswith("mmk::k_conv"):
            continue
        m = {c: statistics.median(v) for c, v in per[k].items()}
        w = m.get("SQ_WAVES") or 1.0
        wc = m.get("SQ_WAVE_CYCLES") or 1.0
        lds = m.get("SQ_ACTIVE_INST_LDS", 0.0)
        out.append("%-30s %6d %6.0f %5.0f %5.0f %6.1f %8.2f %8s %6.3f %6.3f %6.3f" % (
            k[:30], w, m.get("SQ_INSTS_VALU", 0.0) / w, m.get("SQ_INSTS_MFMA", 0.0) / w,
            m.get("SQ_INSTS_LDS", 0.0) / w, m.get("SQ_INSTS_VMEM_RD", 0.0) / w,
            m.get("SQ_VALU_MFMA_BUSY_CYCLES", 0.0) / 1024 / 2400.0,
            "%.3f" % (m.get("SQ_LDS_BANK_CONFLICT", 0.0) / lds) if lds else "-",
            m.get("SQ_WAIT_INST_ANY", 0.0) / wc, m.get("SQ_WAIT_ANY", 0.0) / wc, m.get("SQ_ACTIVE_INST_ANY", 0.0) / wc))
    return "\n".join(out) + "\n"


def table1_euler(torch, mm, W):
    """Per-step time with explicit Euler on N^3 cubes, N = 8 ... 128 (the shape
    of the paper's Table 1; material of the cube workload)."""
    out = []
    for n in (8, 16, 32, 64, 128):
        wl = W.cube(n)
        m = wl.mat
        plan = mm.Plan(n, n, n, *wl.cell)
        plan.autotune(reps=3)
        p = mm.LLGParams.make(Ms=m.Ms, A=m.A, Ku=m.Ku, axis=m.axis, alpha=m.alpha, gamma0=m.gamma0,
                              dt=m.dt, integrator="euler")
        M = torch.from_numpy((m.Ms * wl.initial_unit()).astype("float32")).cuda()
        plan.step(p, M, 5)
        torch.cuda.synchronize()
        k = 200 if n <= 64 else 50
        t0 = time.perf_counter()
        plan.step(p, M, k)
        torch.cuda.synchronize()
        out.append({"N": n, "euler_ms_per_step": (time.perf_counter() - t0) / k * 1e3})
        plan.close()
    return out


def relax_sweep(torch, mm, W, sizes=(8, 16, 32, 64), tol=1e3, max_steps=120000, check_every=250, dt=5e-14):
    """The structure of the paper's cube benchmark (relaxation of N^3 cubes
    with uniaxial anisotropy to the minimum-energy state): mm_llg_relax on
    cubes of the cube workload's material with alpha 1, from a state along
    the easy axis tilted per cell by up to 5 degrees (seeded), until
    max |M x H_eff| / Ms <= tol; steps, time and final observables."""
    import numpy as np
    out = []
    for n in sizes:
        wl = W.cube(n)
        m = wl.mat
        plan = mm.Plan(n, n, n, *wl.cell)
        p = mm.LLGParams.make(Ms=m.Ms, A=m.A, Ku=m.Ku, axis=m.axis, alpha=1.0, gamma0=m.gamma0, dt=dt)
        u0 = W.tilted_unit(n, n, n, seed=600 + n, direction=tuple(m.axis), max_deg=5.0)
        M = torch.from_numpy((m.Ms * u0).astype("float32")).cuda()
        e0 = plan.reduce(p, M)["E_tot"]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = plan.relax(p, M, torque_tol=tol, max_steps=max_steps, check_every=check_every)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        out.append({"N": n, "steps": st["steps"], "seconds": el, "converged": st["torque_max"] <= tol,
                    "torque_max_A_per_m": st["torque_max"], "E_start_J": e0, "E_final_J": st["E_tot"],
                    "m_avg": st["m_avg"]})
        plan.close()
    return {"material": "cube workload (Ms 1e6, A 1.5e-11, Ku 5e4 along x, 2 nm cells), alpha 1, dt %g" % dt,
            "start": "easy axis tilted per cell by up to 5 degrees (seed 600+N)",
            "torque_tol_A_per_m": tol, "check_every": check_every, "rows": out}


def other_configs(torch, mm, W):
    """RK4 step and isolated demag times of the other grid sizes of the
    throughput table (64^3 and 256^3 cubes) and of the learned-form film
    (256x256x4), each with its own autotuned tiles; the step roofline uses
    the same algorithmic bytes as the headline line."""
    out = {}
    for wl, steps in ((W.cube(64), 40), (W.cube(256), 10), (W.film256(0), 40)):
        m = wl.mat
        nx, ny, nz = wl.shape
        plan = mm.Plan(nx, ny, nz, *wl.cell)
        tiles = plan.autotune(reps=3)
        p = mm.LLGParams.make(Ms=m.Ms, A=m.A, Ku=m.Ku, axis=m.axis, alpha=m.alpha, gamma0=m.gamma0,
                              Hext=m.Hext, dt=m.dt)
        M = torch.from_numpy((m.Ms * wl.initial_unit()).astype("float32")).cuda()
        H = torch.empty_like(M)
        plan.step(p, M, 3)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.step(p, M, steps)
        torch.cuda.synchronize()
        st = (time.perf_counter() - t0) / steps
        for _ in range(5):
            plan.demag(M, H)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(50):
            plan.demag(M, H)
        torch.cuda.synchronize()
        dm = (time.perf_counter() - t0) / 50
        b = pass_bytes(nx, ny, nz)
        sbytes = step_bytes(nx, ny, nz, fused=tiles.get("xstage", 0) > 0)
        demag_bytes = sum(v for k, v in b.items() if k not in ("stage", "xstage"))
        out[wl.name] = {"grid": [nx, ny, nz], "ms_per_step": st * 1e3,
                        "cell_updates_per_s": nx * ny * nz / st,
                        "step_roofline_frac": sbytes / st / 1e9 / HBM_PEAK_GBS,
                        "demag_ms": dm * 1e3, "demag_roofline_frac": demag_bytes / dm / 1e9 / HBM_PEAK_GBS,
                        "tiles": tiles}
        plan.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="cube128")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-other-configs", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true")
    ap.add_argument("--summarize-traffic", nargs=2, metavar=("WORKLOAD", "PMC_DIR"),
                    help="print the traffic summary of rocprofv3 counter databases and exit")
    ap.add_argument("--summarize-counters", nargs=3, metavar=("WORKLOAD", "PMC_DIR", "TRACE_DB"),
                    help="print the SQ counter summary of two rocprofv3 --pmc databases (SQ_SETS) and exit")
    ap.add_argument("--summarize-trace", nargs=2, metavar=("WORKLOAD", "DB"),
                    help="print the per-(pass, tile) summary of a rocprofv3 kernel-trace database and exit")
    ap.add_argument("--surrogate-profile", action="store_true",
                    help="run only the learned form's profiled launches (for rocprofv3)")
    ap.add_argument("--summarize-surrogate", metavar="DB",
                    help="print profiles/surrogate_film256.txt from a kernel-trace database")
    ap.add_argument("--summarize-surrogate-counters", metavar="PMC_DIR",
                    help="print profiles/sq_surrogate_film256.txt from the two --pmc runs under PMC_DIR")
    ap.add_argument("--sweep-tiles", action="store_true",
                    help="run only five demag evaluations with every valid tile of every pass "
                         "(for per-tile hardware counters)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run only a plain elementwise copy of 512 MiB (known traffic) for "
                         "scaling the FETCH_SIZE / WRITE_SIZE counters")
    args = ap.parse_args()
    if args.summarize_traffic:
        sys.stdout.write(summarize_traffic(*args.summarize_traffic))
        return
    if args.summarize_surrogate:
        sys.stdout.write(summarize_surrogate(args.summarize_surrogate))
        return
    if args.summarize_surrogate_counters:
        sys.stdout.write(summarize_surrogate_counters(args.summarize_surrogate_counters))
        return
    if args.summarize_trace:
        sys.stdout.write(summarize_trace(*args.summarize_trace))
        return
    if args.summarize_counters:
        sys.stdout.write(summarize_counters(*args.summarize_counters))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU; the library has no multi-GPU path (got --gpus %d)"
              % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1406_7459_amd import mm
    from paper_1406_7459_amd import workloads as W

    if args.calibrate_copy:
        n = 128 * 1024 * 1024  # floats: 512 MiB read + 512 MiB written per launch
        a = torch.ones(n, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            torch.mul(a, 1.0, out=b)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "elementwise copy", "bytes_read_per_launch": 4 * n,
                          "bytes_written_per_launch": 4 * n, "launches": 5}))
        return
    if args.surrogate_profile:
        surrogate_profile(torch, mm)
        print(json.dumps({"surrogate_profile": "film256", "evaluations": 20, "training_steps": 10}))
        return

    name = args.workload
    if name.startswith("cube"):
        wl = W.cube(int(name[4:]))
    elif name == "film256":
        wl = W.film256()
    elif name == "film128":
        wl = W.film128()
    else:
        wl = W.film32()
    nx, ny, nz = wl.shape
    m = wl.mat
    torch.cuda.init()
    t0 = time.perf_counter()
    plan = mm.Plan(nx, ny, nz, *wl.cell)
    setup_s = time.perf_counter() - t0
    if args.sweep_tiles:
        Mw = torch.from_numpy((m.Ms * wl.initial_unit()).astype("float32")).cuda()
        Hw = torch.empty_like(Mw)
        dflt = plan.info()["tiles"]
        done = []
        for pname in ("xfwd", "yfwd", "zconv", "yinv", "xinv", "yconv"):
            if not dflt.get(pname):
                continue
            for tile in [P + 256 * v for v in (0, 1, 2, 3, 4) for P in (1, 2, 4, 8, 16, 32, 64, 128)]:
                try:
                    plan.set_tile(pname, tile)
                except mm.MMError:
                    continue
                for _ in range(5):
                    plan.demag(Mw, Hw)
                done.append("%s.%d" % (pname, tile))
            plan.set_tile(pname, dflt[pname])
        pw = mm.LLGParams.make(Ms=m.Ms, A=m.A, Ku=m.Ku, axis=m.axis, alpha=m.alpha,
                               gamma0=m.gamma0, Hext=m.Hext, dt=m.dt)
        plan.set_tile("xstage", 0)
        for _ in range(3):
            plan.step(pw, Mw, 1)  # the four RK4 stage kernels, launched directly
        for P in [P + 256 * w for w in (0, 1, 2) for P in (1, 2, 4, 8, 16, 32, 64)]:
            try:
                plan.set_tile("xstage", P)
            except mm.MMError:
                continue
            for _ in range(3):
                plan.step(pw, Mw, 1)  # the four fused launches of a step
            done.append("xstage.%d" % P)
        plan.set_tile("xstage", dflt["xstage"])
        torch.cuda.synchronize()
        print(json.dumps({"sweep": name, "tiles": done}))
        return
    tiles = plan.autotune(reps=5) if not args.no_autotune else plan.info()["tiles"]
    params = mm.LLGParams.make(Ms=m.Ms, A=m.A, Ku=m.Ku, axis=m.axis, alpha=m.alpha,
                               gamma0=m.gamma0, Hext=m.Hext, dt=m.dt)
    M = torch.from_numpy((m.Ms * wl.initial_unit()).astype("float32")).cuda()
    stream = torch.cuda.current_stream()

    # warm-up; timed region 1: K RK4 steps replayed from the captured step
    # graph (the value); timed region 2: the same K steps launched directly,
    # every launch bracketed by HIP events on its stream (kernel durations)
    plan.step(params, M, args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.step(params, M, args.steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    plan.set_timing(True)
    plan.timing()  # reset
    t1 = time.perf_counter()
    plan.step(params, M, args.steps)
    torch.cuda.synchronize()
    el_events = time.perf_counter() - t1
    per_kernel = plan.timing()
    plan.set_timing(False)
    st = plan.reduce(params, M)

    # the fused stage pass against the unfused path (x inverse, stage kernel,
    # x forward), both from graph replays, in interleaved rounds
    schedules = {}
    for t in (tiles.get("xstage", 0), 0, 2, 1):
        try:
            plan.set_tile("xstage", t)
        except mm.MMError:
            continue
        schedules.setdefault(t, 1e30)
    Ms = M.clone()
    for _ in range(3):
        for t in schedules:
            plan.set_tile("xstage", t)
            plan.step(params, Ms, 2)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            plan.step(params, Ms, args.steps)
            torch.cuda.synchronize()
            schedules[t] = min(schedules[t], (time.perf_counter() - t1) / args.steps * 1e3)
    plan.set_tile("xstage", tiles.get("xstage", 0))
    del Ms

    # isolated demag evaluations, graph-free, events around the loop
    H = torch.empty_like(M)
    for _ in range(5):
        plan.demag(M, H)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    nd = 100
    for _ in range(nd):
        plan.demag(M, H)
    e1.record(stream)
    torch.cuda.synchronize()
    demag_ms = e0.elapsed_time(e1) / nd

    # Euler steps on the same cube (the integrator of the paper's Table 1)
    pe = mm.LLGParams.make(Ms=m.Ms, A=m.A, Ku=m.Ku, axis=m.axis, alpha=m.alpha,
                           gamma0=m.gamma0, Hext=m.Hext, dt=m.dt, integrator="euler")
    Me = M.clone()
    plan.step(pe, Me, 3)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    plan.step(pe, Me, args.steps)
    torch.cuda.synchronize()
    euler_ms = (time.perf_counter() - t1) / args.steps * 1e3

    bytes_per = pass_bytes(nx, ny, nz)
    fused = tiles.get("xstage", 0) > 0
    sbytes = step_bytes(nx, ny, nz, fused)
    kern = {}
    for k, (ms, n) in per_kernel.items():
        if n > 0:
            kern[k] = dict(launches=n, avg_us=ms / n * 1e3,
                           gbs=(bytes_per.get(k, 0) / (ms / n * 1e-3) / 1e9) if k in bytes_per else None)
    dom = max((k for k in kern if k in bytes_per), key=lambda k: kern[k]["avg_us"] * kern[k]["launches"])
    ach = kern[dom]["gbs"]
    traffic = read_traffic(name, dom, tiles[dom])
    err, nobs = oracle_error_sample(plan, wl, torch)
    cells = nx * ny * nz
    out = {
        "metric": "cell-updates/s",
        "value": cells * args.steps / el,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el / args.steps * 1e3,
        "ms_per_step_event_bracketed_launches": el_events / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": name, "grid": [nx, ny, nz],
                   "padded_fft_grid": [2 * nx, 2 * ny, 2 * nz if nz > 1 else 2],
                   "cell_m": list(wl.cell), "integrator": "rk4", "dt_s": m.dt,
                   "demag_evals_per_step": 4},
        "demag_evals_per_s": 1e3 / demag_ms,
        "demag_ms": demag_ms,
        "demag_roofline_frac": sum(v for k, v in bytes_per.items() if k not in ("stage", "xstage"))
                               / (demag_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "euler_ms_per_step": euler_ms,
        "euler_cell_updates_per_s": cells / (euler_ms * 1e-3),
        "oracle_err": {"H_demag_rel_l2": err, "bar": 1e-5,
                       "sample": "32 random unit sources x Ms at full grid size, %d observer cells "
                                 "(sources included), oracle direct O(N^2) sum" % nobs},
        "state_after": {"E_tot_J": st["E_tot"], "m_avg": st["m_avg"], "nonfinite": st["nonfinite"]},
        "kernels": kern,
        "tiles": tiles,
        "tile_schedules": describe_tiles(tiles),
        "setup_s": setup_s,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": ach, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": ach / HBM_PEAK_GBS, "traffic": traffic,
                     "algorithmic_bytes_per_launch": bytes_per[dom]},
        "step_roofline": {
            "schedule": "fused" if fused else "unfused",
            "algorithmic_bytes_per_step": sbytes,
            "achieved_GBs": sbytes / (el / args.steps) / 1e9,
            "unfused_schedule_bytes_per_step": step_bytes(nx, ny, nz, fused=False),
        },
        "stage_schedules_ms_per_step": {("fused tile %d" % t if t else "unfused"): v for t, v in schedules.items()},
        "paper_context": {"table1_128cube_euler_ms_HD7970_fp32": 26.34,
                          "note": "paper Table 1, Euler, AMD HD 7970, other hardware: context only"},
    }
    out["step_roofline"]["frac"] = out["step_roofline"]["achieved_GBs"] / HBM_PEAK_GBS
    out["table1_shape_euler"] = {
        "rows": table1_euler(torch, mm, W),
        "paper_gpu_ms_HD7970": {"8": 1.95, "16": 2.723, "32": 3.151, "64": 6.558, "128": 26.34},
        "note": "paper Table 1 (Euler, FP32, AMD HD 7970): other hardware, context only"}
    if not args.no_other_configs:
        out["other_configs"] = other_configs(torch, mm, W)
        out["relax_sweep"] = relax_sweep(torch, mm, W)
    if not args.no_batch:
        out["batched"] = batch_measure(torch, mm, W)
    if not args.no_surrogate:
        out["surrogate"] = surrogate_measure(torch, mm, W)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
