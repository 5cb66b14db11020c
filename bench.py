#!/usr/bin/env python
"""Benchmark of the grid-index hot path on one MI355X.

One step = one pass of the whole path over the large ALS tile (10 M points
over 1 km x 1 km, every point a query): build the index (bounding box, voxel
keys, counting-sort reordering, dense voxel map, 1 m cells), plan the query
order, then fixed-radius search (count + prefix sum + fill) at r = 0.5, 1, 2
and 3 m and k-NN at k = 8, 16 and 32.  Inputs are resident in HBM before the
timed region; each call's results are produced in full (CSR neighbour lists,
[Q,k] indices and squared distances).

Prints one JSON line.  ``value`` is queries answered per second over the
whole step (7 query batches of N queries, index build included).  After the
timed steps, one step per voxel map (dense, sparse, mixed) is reported as
the flavor comparison, then the cube and cylinder kernels per radius and
k-NN with Alg. 2's density-growth schedule.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "radius/k-NN queries per sec at 1 GPU; achieved HBM GB/s vs peak; build Mpts/s"
PEAK_HBM_GBS = 8000.0
KERNEL_SOURCES = ["paper_2502_11602_amd/csrc/radius.hip", "paper_2502_11602_amd/csrc/search_common.h",
                  "paper_2502_11602_amd/csrc/common.h"]


def code_text(src):
    """Kernel source without // comments and with whitespace collapsed: the
    part that decides the compiled code."""
    import re

    lines = [re.sub(r"//.*$", "", ln) for ln in src.split("\n")]
    return " ".join(" ".join(lines).split())


def source_hash():
    """Hash of the kernel sources' code (comment edits keep it)."""
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), encoding="utf-8") as fh:
            h.update(code_text(fh.read()).encode())
    return h.hexdigest()[:16]


def counter_traffic(radius):
    """HBM bytes per launch of the radius fill at ``radius`` from the
    committed rocprofv3 PMC summary, or None when there is none or the kernel
    sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "radius_fill_als10m_pmc.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    if d.get("source_hash") != source_hash():
        return None
    return d.get("per_launch_bytes", {}).get(f"fill@r={radius}")


# rocprofv3 runs whose summaries are committed under profiles/ (run from the
# repository root, after `cd /tmp && export TMPDIR=/tmp`, with R the root)
PROFILE_RUNS = {
    "agg": "rocprofv3 --kernel-trace --stats -d $R/gpurun_out/prof_agg -o agg -- "
           "python3 $R/bench.py --workload agg --steps 2",
    "tls": "rocprofv3 --kernel-trace --stats -d $R/gpurun_out/prof_tls -o tls -- "
           "python3 $R/bench.py --workload tls --steps 1 --warmup 0",
    "stats": "rocprofv3 --kernel-trace --stats -d $R/gpurun_out/prof_stats -o stats -- "
             "python3 $R/bench.py --steps 5 --warmup 2 --no-cpu-baseline --no-flavor-compare "
             "--no-kernel-compare",
}
# one step under each counter set (rocprofv3 collects each set in a run of
# its own); the 1 GiB copy calibrates FETCH_SIZE / WRITE_SIZE
PMC_SETS = {
    "fetch": "FETCH_SIZE",
    "write": "WRITE_SIZE",
    "insts": ("SQ_INSTS_VALU SQ_INSTS_SALU SQ_INSTS_LDS SQ_INSTS_VMEM_RD SQ_INSTS_VMEM_WR "
              "SQ_WAVES SQ_WAVE_CYCLES SQ_WAIT_ANY"),
    "busy": ("SQ_ACTIVE_INST_VALU SQ_ACTIVE_INST_LDS SQ_LDS_BANK_CONFLICT SQ_ACTIVE_INST_SCA "
             "SQ_BUSY_CYCLES GRBM_GUI_ACTIVE"),
}
for _k, _c in PMC_SETS.items():
    PROFILE_RUNS[_k] = (f"rocprofv3 --pmc {_c} --kernel-trace -d $R/gpurun_out/prof_{_k} -o {_k} -- "
                        "python3 $R/bench.py --steps 1 --warmup 0 --no-cpu-baseline "
                        "--no-flavor-compare --no-kernel-compare --copy-calibration-mib 1024")
COPY_KERNEL = "__amd_rocclr_copyBuffer"
N_CU = 256
N_XCD = 8  # GRBM_GUI_ACTIVE is summed over the XCDs


def _db(d):
    import glob
    import sqlite3
    f = sorted(glob.glob(os.path.join(d, "**", "*.db"), recursive=True))
    if not f:
        raise SystemExit(f"no rocprofv3 database under {d}")
    return sqlite3.connect(f[0])


def _dispatches(con):
    """(name, duration ms) of every kernel dispatch, in dispatch order."""
    q = ("select S.display_name, K.start, K.end from rocpd_kernel_dispatch K join "
         "rocpd_info_kernel_symbol S on S.id = K.kernel_id and S.guid = K.guid order by K.start")
    return [(n, (e - b) / 1e6) for n, b, e in con.execute(q)]


def _counters(con):
    """[(kernel name, {counter: value summed over instances})] in dispatch order."""
    q = ("select dispatch_id, kernel_name, counter_name, sum(value) from counters_collection "
         "group by dispatch_id, counter_name order by dispatch_id")
    out = {}
    for d, n, c, v in con.execute(q):
        out.setdefault(d, (n, {}))[1][c] = v
    return [out[d] for d in sorted(out)]


def _second_launch(name):
    """The second launch of a ring k-NN or radius-tile search (the waves the
    first listed, template argument CL = 2), which the per-kernel table
    shows on its own."""
    n = name.replace(" ", "")
    return (("k_knn<" in n and n.endswith(",2>(chs::KnnArgs)")) or
            ("k_radius_tile<" in n and n.endswith(",2>(chs::RadiusArgs)")))


def _knn_first(name):
    """A ring k-NN launch other than the second one of a search."""
    return "k_knn<" in name and not _second_launch(name)


def _hot_kernels(seq, radii, ks):
    """Label the search launches of one bench step, in their order: the count
    and fill of each radius, then k-NN per k.  seq: [(name, payload)]."""
    counts = [x for x in seq if "k_radius" in x[0] and "<false" in x[0] and not _second_launch(x[0])]
    fills = [x for x in seq if "k_radius" in x[0] and "<true" in x[0] and not _second_launch(x[0])]
    knns = [x for x in seq if _knn_first(x[0])]
    lab = []
    for i, r in enumerate(radii):
        lab.append((f"count r={r:g}", counts[i]))
        lab.append((f"fill r={r:g}", fills[i]))
    for i, k in enumerate(ks):
        lab.append((f"knn k={k}", knns[i]))
    return lab


def agg_profile_summary(stats_dir):
    """Write the committed kernel-time summary of the aggregation workload."""
    disp = _dispatches(_db(stats_dir))
    agg = {}
    for name, ms in disp:
        a = agg.setdefault(name, [0, 0.0])
        a[0] += 1
        a[1] += ms
    total = sum(v[1] for v in agg.values())
    lines = ["# Kernel times, Gaussian aggregation workload (1 M points, 250 k centres, "
             "64 channels)", "",
             "Command (from the repository root R, after `cd /tmp && export TMPDIR=/tmp`):", "",
             "    " + PROFILE_RUNS["agg"], "",
             "Neighbour lists (k-NN, 64 nearest within 0.5 m) plus three forward and three "
             "forward + backward passes per feature type (FP32, then BF16), the first of each a "
             "warm-up.  Per kernel: dispatches, total and average duration.", "",
             "| kernel | calls | total ms | avg ms | % |", "|---|---:|---:|---:|---:|"]
    for name, (c, ms) in sorted(agg.items(), key=lambda kv: -kv[1][1])[:20]:
        lines.append(f"| `{name[:90]}` | {c} | {ms:.3f} | {ms / c:.4f} | {100 * ms / total:.1f} |")
    out_dir = os.path.join(ROOT, "profiles")
    os.makedirs(out_dir, exist_ok=True)
    with open(os.path.join(out_dir, "gauss_agg_1m.md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print(json.dumps({"kernels": len(agg)}))


def tls_profile_summary(stats_dir, bench_log):
    """Write the committed summary of the TLS workload: kernel times from the
    rocprofv3 run and the bench line that run printed."""
    disp = _dispatches(_db(stats_dir))
    agg = {}
    for name, ms in disp:
        a = agg.setdefault(name, [0, 0.0])
        a[0] += 1
        a[1] += ms
    total = sum(v[1] for v in agg.values())
    res = None
    with open(bench_log) as fh:
        for line in fh:
            if line.startswith('{"metric"'):
                res = json.loads(line)
    lines = ["# TLS scan: 20 M points, 2 M query points, 0.25 m voxels (MI355X)", "",
             "Command (from the repository root R, after `cd /tmp && export TMPDIR=/tmp`):", "",
             "    " + PROFILE_RUNS["tls"], "",
             "Per flavor (sparse, then mixed): the queries put in the searches' processing "
             "order; per radius one count pass under each schedule (the faster is kept), then "
             "the timed count over all queries and the fill range by range (at most %d "
             "entries per range); then k-NN with k = 32." % (res or {}).get("chunk_entries", 0),
             ""]
    if res:
        lines += ["| flavor | r (m) | schedule | neighbours | ranges | count ms | fill ms | "
                  "neighbours/s |", "|---|---|---|---:|---:|---:|---:|---:|"]
        for fl, rec in res["flavors"].items():
            for r, v in rec["radius"].items():
                lines.append(f"| {fl} | {r} | {v['schedule']} | {v['neighbours']:.3e} | "
                             f"{v['ranges']} | {v['count_ms']:.1f} | {v['chunked_fill_ms']:.1f} | "
                             f"{v['neighbours_per_s']:.2e} |")
        lines += ["", "k-NN (k = 32, 2 M queries): " + ", ".join(
            f"{fl} {rec['knn']['ms']:.1f} ms" for fl, rec in res["flavors"].items()),
            "", f"Whole job: {res['value']:.3e} neighbours/s ({res['ms_per_step']:.0f} ms for "
            "the three radii of the faster flavor).", ""]
    lines += ["Kernel dispatches of the whole run (both flavors, schedule trials included):",
              "", "| kernel | calls | total ms | avg ms | % |", "|---|---:|---:|---:|---:|"]
    for name, (c, ms) in sorted(agg.items(), key=lambda kv: -kv[1][1])[:16]:
        lines.append(f"| `{name[:90]}` | {c} | {ms:.3f} | {ms / c:.4f} | {100 * ms / total:.1f} |")
    out_dir = os.path.join(ROOT, "profiles")
    with open(os.path.join(out_dir, "tls_scan_20m.md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print(json.dumps({"kernels": len(agg)}))


def profile_summary(stats_dir, pmc_root, radii=(0.5, 1.0, 2.0, 3.0), ks=(8, 16, 32),
                    n=10_000_000):
    """Write the committed rocprofv3 summaries of the default step (10 M-point
    ALS tile): per-kernel times; per search launch the instruction mix,
    LDS bank conflicts, waits and HBM bytes per query; and the HBM traffic of
    the r = 3 m fill (FETCH_SIZE / WRITE_SIZE scaled by what the counters read
    for a 1 GiB device copy).  pmc_root holds prof_<set> for every PMC set."""
    out_dir = os.path.join(ROOT, "profiles")
    os.makedirs(out_dir, exist_ok=True)
    # ---- kernel times
    disp = _dispatches(_db(stats_dir))
    agg = {}
    for name, ms in disp:
        a = agg.setdefault(name, [0, 0.0])
        a[0] += 1
        a[1] += ms
    total = sum(v[1] for v in agg.values())
    steps = 7  # 2 warm-up + 5 timed
    lab = {}
    # the labelled launches of every step, averaged over the steps
    counts = [(nm, ms) for nm, ms in disp
              if "k_radius" in nm and "<false" in nm and not _second_launch(nm)]
    fills = [(nm, ms) for nm, ms in disp
             if "k_radius" in nm and "<true" in nm and not _second_launch(nm)]
    knns = [(nm, ms) for nm, ms in disp if _knn_first(nm)]
    for i, r in enumerate(radii):
        c = counts[i::len(radii)]
        f = fills[i::len(radii)]
        lab[f"count r={r:g}"] = (c[0][0], sum(m for _, m in c) / len(c))
        lab[f"fill r={r:g}"] = (f[0][0], sum(m for _, m in f) / len(f))
    for i, k in enumerate(ks):
        kk = knns[i::len(ks)]
        lab[f"knn k={k}"] = (kk[0][0], sum(m for _, m in kk) / len(kk))
    lines = ["# Kernel times, default bench step (10 M-point ALS tile)", "",
             "Command (from the repository root R, after `cd /tmp && export TMPDIR=/tmp`):", "",
             "    " + PROFILE_RUNS["stats"], "",
             f"{steps} steps profiled (2 warm-up + 5 timed).  Per kernel: dispatches, total and "
             "average duration.", "",
             "| kernel | calls | total ms | avg ms | % |", "|---|---:|---:|---:|---:|"]
    for name, (c, ms) in sorted(agg.items(), key=lambda kv: -kv[1][1])[:25]:
        lines.append(f"| `{name[:90]}` | {c} | {ms:.3f} | {ms / c:.4f} | {100 * ms / total:.1f} |")
    lines += ["", "Search launches of a step, average ms per launch:", "",
              "| launch | kernel | avg ms |", "|---|---|---:|"]
    for key, (nm, ms) in lab.items():
        lines.append(f"| {key} | `{nm[:70]}` | {ms:.3f} |")
    with open(os.path.join(out_dir, "kernels_als10m.md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    # ---- counters of one step
    pmc = {k: _counters(_db(os.path.join(pmc_root, f"prof_{k}"))) for k in PMC_SETS}

    def copy_kib(seq, counter):
        return max(c.get(counter, 0.0) for nm, c in seq if COPY_KERNEL in nm)

    gib = float(1 << 30)
    f_fac = gib / (copy_kib(pmc["fetch"], "FETCH_SIZE") * 1024.0)
    w_fac = gib / (copy_kib(pmc["write"], "WRITE_SIZE") * 1024.0)
    hot = {k: dict(_hot_kernels(v, radii, ks)) for k, v in pmc.items()}
    rows = []
    rec = {}
    for key in hot["insts"]:
        nm, ci = hot["insts"][key]
        cb = hot["busy"][key][1]
        rd = hot["fetch"][key][1].get("FETCH_SIZE", 0.0) * 1024.0 * f_fac
        wr = hot["write"][key][1].get("WRITE_SIZE", 0.0) * 1024.0 * w_fac
        cyc = cb["GRBM_GUI_ACTIVE"] / N_XCD
        r = dict(kernel=nm, valu_per_query=ci["SQ_INSTS_VALU"] / n,
                 salu_per_query=ci["SQ_INSTS_SALU"] / n, lds_per_query=ci["SQ_INSTS_LDS"] / n,
                 vmem_rd_per_query=ci["SQ_INSTS_VMEM_RD"] / n,
                 vmem_wr_per_query=ci["SQ_INSTS_VMEM_WR"] / n,
                 valu_per_cu_cycle=ci["SQ_INSTS_VALU"] / (N_CU * cyc),
                 salu_per_cu_cycle=ci["SQ_INSTS_SALU"] / (N_CU * cyc),
                 wait_share=ci["SQ_WAIT_ANY"] / max(ci["SQ_WAVE_CYCLES"], 1.0),
                 lds_bank_conflict_share=cb["SQ_LDS_BANK_CONFLICT"] / max(cb["SQ_ACTIVE_INST_LDS"], 1.0),
                 read_bytes=rd, write_bytes=wr, bytes_per_query=(rd + wr) / n, gpu_cycles=cyc)
        rec[key] = r
        rows.append(f"| {key} | {r['valu_per_query']:.1f} | {r['salu_per_query']:.1f} | "
                    f"{r['lds_per_query']:.2f} | {r['valu_per_cu_cycle']:.2f} | "
                    f"{r['salu_per_cu_cycle']:.2f} | {100 * r['wait_share']:.0f} % | "
                    f"{100 * r['lds_bank_conflict_share']:.1f} % | {rd / 1e9:.2f} | {wr / 1e9:.2f} | "
                    f"{r['bytes_per_query']:.0f} |")
    cmds = ["    " + PROFILE_RUNS[k] for k in PMC_SETS]
    md = ["# Counters of the search kernels, one default step (10 M-point ALS tile, every point "
          "a query, dense, 1 m voxels)", "",
          "Commands (from the repository root R, after `cd /tmp && export TMPDIR=/tmp`), one "
          "counter set per run:", ""] + cmds + [
          "", "Summary: `python3 bench.py --profile-summary <stats dir> <dir holding prof_<set>>`.",
          "",
          "Per launch: wave instructions per query (VALU, SALU, LDS), VALU and SALU wave "
          "instructions per CU per GPU cycle (GRBM_GUI_ACTIVE per XCD), the share of wave "
          "cycles spent waiting (SQ_WAIT_ANY / SQ_WAVE_CYCLES), LDS bank-conflict cycles per "
          "active LDS cycle, HBM bytes read and written (FETCH_SIZE x %.4f, WRITE_SIZE x %.4f, "
          "the factors that make a 1 GiB device copy read and write 1 GiB) and bytes per query."
          % (f_fac, w_fac), "",
          "| launch | VALU/q | SALU/q | LDS/q | VALU/CU/cyc | SALU/CU/cyc | waiting | LDS "
          "conflicts | read GB | written GB | B/q |",
          "|---|---:|---:|---:|---:|---:|---:|---:|---:|---:|---:|"] + rows + [
          "", "Kernel sources hash: `%s` (bench.py reports the r = 3 m fill's traffic only "
          "while the code matches)." % source_hash()]
    with open(os.path.join(out_dir, "counters_als10m.md"), "w") as fh:
        fh.write("\n".join(md) + "\n")
    fill3 = rec[f"fill r={radii[-1]:g}"]
    js = {"workload": "10 M-point ALS tile, every point a query, dense, 1 m voxels",
          "commands": {k: PROFILE_RUNS[k] for k in PMC_SETS},
          "calibration": {"fetch_factor": f_fac, "write_factor": w_fac},
          "launches": rec, "source_hash": source_hash(),
          "per_launch_bytes": {f"fill@r={radii[-1]}": fill3["read_bytes"] + fill3["write_bytes"]}}
    with open(os.path.join(out_dir, "radius_fill_als10m_pmc.json"), "w") as fh:
        json.dump(js, fh, indent=1)
    print(json.dumps({"kernels": len(agg), "fill_traffic": js["per_launch_bytes"]}), flush=True)


def cpu_baseline(xyz, radii, ks, cell, sample, nthreads):
    """The oracle as it stands, on the host cores: full build plus a seeded
    sample of queries per radius / k, scaled to the whole step."""
    import numpy as np

    import oracle

    n = xyz.shape[0]
    q = np.sort(np.random.default_rng(99).choice(n, sample, replace=False)).astype(np.int32)
    t0 = time.perf_counter()
    ox = oracle.OracleIndex(xyz, cell)
    t_build = time.perf_counter() - t0
    per_q = 0.0
    for r in radii:
        t0 = time.perf_counter()
        ox.radius(r, pidx=q, nthreads=nthreads)
        per_q += (time.perf_counter() - t0) / sample
    for k in ks:
        t0 = time.perf_counter()
        ox.knn(k, pidx=q, nthreads=nthreads)
        per_q += (time.perf_counter() - t0) / sample
    t_step = t_build + per_q * n
    nops = len(radii) + len(ks)
    return {
        "value": nops * n / t_step,
        "unit": "queries/s",
        "cores": nthreads,
        "kind": "oracle",
        "sample": (f"full oracle build of the {n}-point cloud ({t_build:.1f} s, one thread) plus "
                   f"{sample} seeded point queries per radius and per k on {nthreads} threads, "
                   f"scaled to {n} queries per batch"),
        "build_s": t_build,
        "query_us_per_thread": per_q * 1e6 * nthreads / nops,
    }


def agg_bytes(N, Q, K, C, P, fbytes):
    """Algorithmic HBM bytes of the aggregation passes for Q centres with K
    slots each, P valid (centre, neighbour) pairs, C channels of fbytes bytes:
    every pair reads its neighbour's feature row and coordinates once.
    Forward: rows 4C and x 12 per pair, the lists 4KQ, centres 16Q, output.
    Backward (the sort excluded): the pair pass reads the rows, x and g per
    centre and writes w, s, key and value per slot and the centre gradient;
    the point pass reads per pair the sorted slot, w, s, the centre index,
    its coordinates and g row, and writes the feature and coordinate
    gradients."""
    row = C * fbytes
    fwd = P * (row + 12) + 4 * K * Q + 16 * Q + row * Q
    pairs = P * (row + 12) + row * Q + 4 * K * Q + 16 * K * Q + 8 * Q + 16 * Q
    points = P * (4 + 8 + 4 + 12 + row) + 8 * (N + 1) + 4 * Q + N * (row + 12)
    return fwd, pairs + points


def run_agg(args):
    """Aggregation workload: 1 M ALS-like points at about 50 points per
    square metre, 64-channel N(0, 1) features, 250 k centres drawn from the
    points, neighbour lists of the 64 nearest within 0.5 m, sigma 0.25 m.
    Times the neighbour search, the forward and the backward with FP32 and
    with BF16 features, and reports each pass's bandwidth for its
    algorithmic bytes (agg_bytes) against the HBM peak."""
    import numpy as np
    import torch

    import cloudgen
    from paper_2502_11602_amd import GridIndex, gauss_aggregate, neighbour_lists
    from paper_2502_11602_amd.agg import recentred
    from paper_2502_11602_amd.autotune import pick_knn_schedule

    c = cloudgen.config4()
    dev = torch.device("cuda:0")
    x64 = torch.from_numpy(c["xyz"]).to(dev)
    q = torch.from_numpy(c["queries"]).to(dev)
    f32 = torch.from_numpy(c["f"]).to(dev)
    N, C = f32.shape
    Q, K, sigma = q.numel(), c["k"], c["sigma"]
    E = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731

    def timed(fn, reps):
        ts = []
        for _ in range(reps):
            a, b = E(), E()
            a.record()
            fn()
            b.record()
            torch.cuda.synchronize()
            ts.append(a.elapsed_time(b))
        return sum(ts[1:]) / max(1, len(ts) - 1)  # the first is a warm-up

    reps = max(2, args.steps + 1)
    ix = GridIndex(x64, cell=args.agg_cell, flavor="dense")
    # the k-NN schedule of these lists, by timing both (a quarter of the
    # points as centres: one query at a time usually wins)
    knn_sched, knn_sched_ms = pick_knn_schedule(ix, K, q, r_max=c["r"])
    nbr = neighbour_lists(ix, q, k=K, r_max=c["r"])
    t_nbr = timed(lambda: neighbour_lists(ix, q, k=K, r_max=c["r"]), reps)
    x32 = recentred(ix)
    P = int((nbr >= 0).sum())
    res = {}
    for name, dt in (("f32", torch.float32), ("bf16", torch.bfloat16)):
        f = f32.to(dt)
        g = torch.randn((Q, C), generator=torch.Generator().manual_seed(3)).to(dev).to(dt)
        with torch.no_grad():
            t_fwd = timed(lambda: gauss_aggregate(x32, f, q, nbr, sigma=sigma), reps)
        xg = x32.clone().requires_grad_(True)
        fg = f.clone().requires_grad_(True)

        def fwd_bwd():
            xg.grad = None
            fg.grad = None
            out = gauss_aggregate(xg, fg, q, nbr, sigma=sigma)
            out.backward(g)

        t_fb = timed(fwd_bwd, reps)
        t_bwd = t_fb - t_fwd
        fb = 2 if dt == torch.bfloat16 else 4
        bf, bb = agg_bytes(N, Q, K, C, P, fb)
        # the method's minimum: every feature row and coordinate once, the
        # lists, the centres and the output
        bmin = C * fb * N + 12 * (N + Q) + 4 * K * Q + C * fb * Q
        res[name] = {"forward_ms": t_fwd, "backward_ms": t_bwd,
                     "forward_min_bytes": bmin,
                     "forward_min_gbs": bmin / (t_fwd / 1e3) / 1e9,
                     "forward_gbs": bf / (t_fwd / 1e3) / 1e9,
                     "backward_gbs": bb / (t_bwd / 1e3) / 1e9,
                     "forward_bytes": bf, "backward_bytes": bb}
        print(f"[bench] agg {name}: fwd {t_fwd:.3f} ms, bwd {t_bwd:.3f} ms",
              file=sys.stderr, flush=True)
    ix.close()
    f = res["f32"]
    out = {
        "metric": "Gaussian aggregation: centres per sec (forward + backward, FP32 features)",
        "value": Q / ((f["forward_ms"] + f["backward_ms"]) / 1e3),
        "unit": "centres/s",
        "n_gpus": 1, "steps": reps - 1, "warmup": 1,
        "ms_per_step": f["forward_ms"] + f["backward_ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"ALS-like cloud, {N} points at about 50 points/m^2, {Q} centres, "
                               f"{C} channels, {K} nearest within {c['r']} m, sigma {sigma} m",
                   "cell_m": args.agg_cell, "valid_pairs": P},
        "neighbour_lists_ms": t_nbr,
        "neighbour_lists_schedule": knn_sched, "schedule_trials_ms": knn_sched_ms,
        "passes": res,
        # against the method's minimum bytes (features read once); the
        # per-pair gather bytes (a feature row per valid pair) beside it
        "roofline": {"kernel": "k_agg_fwd (f32)", "bound": "hbm",
                     "achieved": f["forward_min_gbs"], "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": f["forward_min_gbs"] / PEAK_HBM_GBS, "traffic": None,
                     "algorithmic_bytes": f["forward_min_bytes"], "launch_ms": f["forward_ms"],
                     "gather": {"bytes": f["forward_bytes"], "achieved": f["forward_gbs"],
                                "frac": f["forward_gbs"] / PEAK_HBM_GBS}},
    }
    print(json.dumps(out), flush=True)


def run_batched(args):
    """Batched workload: 256 ALS-like tiles, sizes log-uniform in 1e4..2e6
    (about 60 M points), densities 2-20 points per square metre; every point
    queries its own tile with r = 1 m and k = 16.  Voxel edges per tile come
    from the autotuner.  Times one batched build + persistent searches (and
    the searches replayed from a hipGraph) against 256 per-tile index builds
    and launch sequences, and checks both give identical results."""
    import numpy as np
    import torch

    import cloudgen
    from paper_2502_11602_amd import GridIndex
    from paper_2502_11602_amd.autotune import Autotuner

    r, k = args.batch_r, args.batch_k
    nt, dens, tile_cloud = cloudgen.config3_tiles(scale=args.batch_scale)
    T = len(nt)
    print(f"[bench] generating {T} tiles, {int(nt.sum())} points", file=sys.stderr, flush=True)
    tiles_np = [tile_cloud(t) for t in range(T)]
    frames = [list(t.min(0)) + list(t.max(0)) for t in tiles_np]
    toff = np.concatenate([[0], np.cumsum([len(t) for t in tiles_np])]).astype(np.int64)
    dev = torch.device("cuda:0")
    x = torch.from_numpy(np.concatenate(tiles_np)).to(dev)
    del tiles_np
    tiles = [x[toff[t]:toff[t + 1]] for t in range(T)]
    n = int(toff[-1])
    tuner = Autotuner(cache_path=args.tune_cache)
    t0 = time.perf_counter()
    cells, flavor, sched = tuner.choose(tiles, r, k)
    tune_s = time.perf_counter() - t0
    print(f"[bench] autotune {tune_s:.1f} s ({len(tuner.trials)} trials), flavor {flavor}, "
          f"radius schedule {sched}", file=sys.stderr, flush=True)
    tuner.save()
    toff_l = toff.tolist()

    def batched(keep=False):
        ix = GridIndex(x, cell=cells, flavor=flavor, tile_off=toff_l)
        ix.set_radius_schedule(sched)
        off, tot = ix.radius_count(r)
        nbr = ix.radius_fill(r, off, tot)
        idx, d2 = ix.knn(k)
        return (ix, off, tot, nbr, idx, d2) if keep else None

    def per_tile(keep=False):
        res = []
        for t in range(T):
            ix = GridIndex(tiles[t], cell=cells[t], flavor=flavor)
            ix.set_radius_schedule(sched)
            off, tot = ix.radius_count(r)
            nbr = ix.radius_fill(r, off, tot)
            idx, d2 = ix.knn(k)
            if keep:
                res.append((off, nbr, idx, d2))
            ix.close()
        return res

    def timed(fn, steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    # identical results: batched rows equal the per-tile rows (same order)
    ix, off, tot, nbr, idx, d2 = batched(keep=True)
    pt = per_tile(keep=True)
    same = True
    for t in range(T):
        a, b = toff[t], toff[t + 1]
        o_b = off[a:b + 1] - off[a]
        o_t, n_t, i_t, d_t = pt[t]
        same &= bool(torch.equal(o_b, o_t))
        same &= bool(torch.equal(nbr[int(off[a]):int(off[b])], n_t))
        same &= bool(torch.equal(idx[a:b], i_t)) and bool(torch.equal(d2[a:b], d_t))
    del pt
    print(f"[bench] batched == per-tile: {same}", file=sys.stderr, flush=True)
    # hipGraph of the searches on the batched index
    nbr_g = torch.empty_like(nbr)
    idx_g = torch.empty_like(idx)
    d2_g = torch.empty_like(d2)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        ix.radius_fill(r, off, tot, out=nbr_g)
        ix.knn_into(k, idx_g, d2_g)
    torch.cuda.current_stream().wait_stream(s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        ix.radius_fill(r, off, tot, out=nbr_g)
        ix.knn_into(k, idx_g, d2_g)
    g.replay()
    torch.cuda.synchronize()
    same_graph = bool(torch.equal(nbr_g, nbr)) and bool(torch.equal(idx_g, idx)) \
        and bool(torch.equal(d2_g, d2))
    # the whole step as two graphs: A = build from the tiles' frames + count
    # (nothing read back), one read of the total, B = fill + k-NN
    off_a = torch.empty(n + 1, dtype=torch.int64, device=dev)
    nbr_b = torch.empty_like(nbr)
    idx_b = torch.empty_like(idx)
    d2_b = torch.empty_like(d2)
    with torch.cuda.stream(s):
        wix = GridIndex(x, cell=cells, flavor=flavor, tile_off=toff_l, frames=frames)
        wix.set_radius_schedule(sched)
        wix.radius_count(r, sync=False, out=off_a)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    del wix
    ga = torch.cuda.CUDAGraph()
    with torch.cuda.graph(ga):
        gix = GridIndex(x, cell=cells, flavor=flavor, tile_off=toff_l, frames=frames)
        gix.set_radius_schedule(sched)
        gix.radius_count(r, sync=False, out=off_a)
    ga.replay()
    torch.cuda.synchronize()
    tot_a = int(off_a[-1])
    with torch.cuda.stream(s):
        gix.radius_fill(r, off_a, tot_a, out=nbr_b)
        gix.knn_into(k, idx_b, d2_b)
    torch.cuda.current_stream().wait_stream(s)
    gb = torch.cuda.CUDAGraph()
    with torch.cuda.graph(gb):
        gix.radius_fill(r, off_a, tot_a, out=nbr_b)
        gix.knn_into(k, idx_b, d2_b)

    def graphs():
        ga.replay()
        t = int(off_a[-1])  # the one read between the graphs
        assert t == tot_a
        gb.replay()

    graphs()
    torch.cuda.synchronize()
    same_graphs = bool(torch.equal(off_a, off)) and bool(torch.equal(nbr_b, nbr)) \
        and bool(torch.equal(idx_b, idx)) and bool(torch.equal(d2_b, d2))
    print(f"[bench] two-graph step == eager: {same_graphs}", file=sys.stderr, flush=True)
    del nbr, idx, d2
    for _ in range(args.warmup):
        batched()
        per_tile()
    t_batch = timed(batched, args.steps)
    t_tile = timed(per_tile, max(1, args.steps // 2))
    t_graph_search = timed(lambda: g.replay(), args.steps)
    t_graphs = timed(graphs, args.steps)
    out = {
        "metric": "batched uneven tiles: queries per sec, one batched launch sequence vs "
                  "per-tile launches",
        "value": 2 * n / t_batch,
        "unit": "queries/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": t_batch * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{T} ALS tiles, {n} points, sizes log-uniform, densities "
                               f"2-20 pts/m2; radius r={r} m + k-NN k={k} per tile; "
                               "autotuned voxel edges", "flavor": flavor,
                   "radius_schedule": sched, "tiles": T,
                   "n_points": n},
        "batched_ms": t_batch * 1e3,
        "per_tile_ms": t_tile * 1e3,
        "speedup_vs_per_tile": t_tile / t_batch,
        "graph_replay_fill_knn_ms": t_graph_search * 1e3,
        "two_graph_step_ms": t_graphs * 1e3,
        "two_graph_speedup_vs_per_tile": t_tile / t_graphs,
        "identical_results": same,
        "graph_identical": same_graph,
        "two_graph_identical": same_graphs,
        "autotune_s": tune_s,
        "cells_m": {"min": min(cells), "max": max(cells)},
    }
    print(json.dumps(out), flush=True)
    if args.write_summary:
        md = ["# Batched uneven tiles: one batched launch sequence, two captured graphs, "
              "per-tile launches (MI355X)", "", "Command (repository root):", "",
              "    python -u bench.py --workload batched --steps %d --warmup %d --write-summary"
              % (args.steps, args.warmup), "",
              f"Workload: {T} ALS-like tiles (sizes log-uniform 1e4..2e6, rescaled to about 60 M "
              f"points; densities 2-20 pts/m^2); every point queries its own tile, radius "
              f"r = {r} m (count + fill) and k-NN k = {k}; voxel edge, flavor and radius schedule "
              f"per tile from the autotuner (edges {min(cells):.3g}-{max(cells):.4g} m; "
              f"{flavor} flavor; schedule `{sched}`).", "",
              "| quantity | value |", "|---|---|",
              f"| n_points | {n} |", f"| tiles | {T} |",
              f"| batched_ms | {t_batch * 1e3:.1f} |", f"| two_graph_step_ms | {t_graphs * 1e3:.1f} |",
              f"| per_tile_ms | {t_tile * 1e3:.1f} |",
              f"| speedup_vs_per_tile | {t_tile / t_batch:.2f} (two graphs: {t_tile / t_graphs:.2f}) |",
              f"| graph_replay_fill_knn_ms | {t_graph_search * 1e3:.2f} |",
              f"| identical_results | {same} |", f"| graph_identical | {same_graph} |",
              f"| two_graph_identical | {same_graphs} |", f"| autotune_s | {tune_s:.1f} |",
              f"| value (queries/s) | {2 * n / t_batch:.3e} |", "",
              "- batched_ms: build + radius count + fill + k-NN for the whole batch (persistent "
              "waves), eager calls;",
              "- two_graph_step_ms: the same step as graph A (build from the tiles' bounding "
              "boxes, which reads nothing back, + count + offsets) replayed, one read of the "
              "neighbour total, then graph B (fill + k-NN) replayed;",
              "- per_tile_ms: the same calls on separate per-tile indexes;",
              "- graph_replay_fill_knn_ms: fill + k-NN replayed from a graph on the eager index;",
              "- every variant's offsets, neighbour rows and k-NN lists equal the per-tile calls' "
              "(`identical_results`, `*_identical`);", "- value = 2 x points / batched_ms."]
        with open(os.path.join(ROOT, "profiles", "batched_tiles_60m.md"), "w") as fh:
            fh.write("\n".join(md) + "\n")


def run_sweep(args):
    """The paper's cell-size study on the 10 M-point ALS tile (Sections 5.1-5.2):
    voxel edges 1, 2.5, 5, 7.5, 10 m x 2D/3D grids x dense/sparse/mixed
    maps.  Per configuration: build time, device bytes per point (the
    paper's minimum is one 8-byte pointer per point), radius search (count +
    fill) at 1 and 3 m and k-NN at k = 16 over every point, one warm and one
    measured pass each."""
    import torch

    import cloudgen
    from paper_2502_11602_amd import GridIndex

    print(f"[bench] generating ALS tile: {args.points} points", file=sys.stderr, flush=True)
    xyz = cloudgen.config1(n=args.points)["xyz"]
    n = xyz.shape[0]
    x = torch.from_numpy(xyz).to(torch.device("cuda:0"))
    torch.cuda.synchronize()
    E = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
    rows = []
    for cell in (1.0, 2.5, 5.0, 7.5, 10.0):
        for dims in (3, 2):
            for fl in ("dense", "sparse", "mixed"):
                rec = {}
                for rep in range(2):
                    ev = [E() for _ in range(5)]
                    ev[0].record()
                    ix = GridIndex(x, cell=cell, dims=dims, flavor=fl)
                    ev[1].record()
                    torch.cuda.synchronize()
                    built = ix.info()["device_bytes"]
                    off, nbr = ix.radius(1.0)
                    ev[2].record()
                    del off, nbr
                    off, nbr = ix.radius(3.0)
                    ev[3].record()
                    del off, nbr
                    idx, d2 = ix.knn(16)
                    ev[4].record()
                    del idx, d2
                    torch.cuda.synchronize()
                    rec = {"cell_m": cell, "dims": dims, "flavor": fl,
                           "build_ms": ev[0].elapsed_time(ev[1]),
                           "radius_1m_ms": ev[1].elapsed_time(ev[2]),
                           "radius_3m_ms": ev[2].elapsed_time(ev[3]),
                           "knn16_ms": ev[3].elapsed_time(ev[4]),
                           "device_bytes_per_point": built / n,
                           "nonempty_voxels": ix.info()["n_nonempty"]}
                    ix.close()
                rows.append(rec)
                print(f"[bench] sweep cell={cell} dims={dims} {fl} done", file=sys.stderr, flush=True)
    best = min(rows, key=lambda r: r["radius_1m_ms"] + r["radius_3m_ms"] + r["knn16_ms"])
    ms = best["build_ms"] + best["radius_1m_ms"] + best["radius_3m_ms"] + best["knn16_ms"]
    out = {"metric": "cell-size x 2D/3D x flavor sweep: best queries/s (build + r=1,3 m + k=16)",
           "value": 3 * n / (ms / 1e3), "unit": "queries/s", "n_gpus": 1, "steps": 1,
           "warmup": 1, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"ALS tile, {n} points, every point a query; voxel edges "
                                  "1-10 m, 2D and 3D grids, dense/sparse/mixed maps",
                      "n_points": n},
           "paper_min_bytes_per_point": 8, "best": best, "rows": rows}
    print(json.dumps(out), flush=True)
    if args.write_summary:
        md = ["# Cell size x 2D/3D x voxel map sweep, 10 M-point ALS tile (MI355X)", "",
              "Command (repository root):", "",
              "    python -u bench.py --workload sweep --write-summary", "",
              "Every point a query; per configuration one warm and one measured pass: build, "
              "radius search (count + fill) at 1 m and 3 m, k-NN at k = 16.  bytes/point is the "
              "index's device memory right after the build (`chs_index_info`) divided by the "
              "point count; the paper's minimum for a pointer-based index is 8 bytes per point, "
              "this index keeps FP32 copies of the cloud in voxel order (16 B float4 + 12 B SoA) "
              "and both permutations (8 B), so 36 B per point, plus the processing order of "
              "every-point queries planned at build time (16 B per point) and the voxel maps "
              "(the sparse and mixed maps: the voxel hash and the column directory).", "",
              "| cell (m) | grid | map | build ms | r=1 m ms | r=3 m ms | k=16 ms | bytes/point | "
              "non-empty voxels |", "|---:|---|---|---:|---:|---:|---:|---:|---:|"]
        for r in rows:
            md.append(f"| {r['cell_m']} | {r['dims']}D | {r['flavor']} | {r['build_ms']:.2f} | "
                      f"{r['radius_1m_ms']:.2f} | {r['radius_3m_ms']:.2f} | {r['knn16_ms']:.2f} | "
                      f"{r['device_bytes_per_point']:.1f} | {r['nonempty_voxels']} |")
        md += ["", f"Fastest searches: {best['cell_m']} m, {best['dims']}D, {best['flavor']} "
               f"(r = 1 m + r = 3 m + k = 16: {best['radius_1m_ms'] + best['radius_3m_ms'] + best['knn16_ms']:.2f} ms)."]
        with open(os.path.join(ROOT, "profiles", "cell_size_sweep_als10m.md"), "w") as fh:
            fh.write("\n".join(md) + "\n")


def run_tls(args):
    """The TLS scan (Section 4.1, Table 1: terrestrial scans, density falling
    with the range from the scanner): 20 M points, 2 M query points drawn
    from the cloud, 0.25 m voxels, sparse and mixed maps.  Per radius (0.1,
    0.25, 0.5 m): the count pass over all 2 M queries, then the fill range by
    range (the queries taken in the searches' processing order, so that each
    range is spatially compact), each range's rows within a budget of
    --chunk-entries neighbour
    entries (one reused buffer; at 0.5 m the relation holds about 1.5e11
    pairs, 600 GB of indices, beyond one GPU's memory).  All tiles of a
    range start at once, so a range lasts as long as its slowest tile: few,
    large ranges (2^35 entries, 128 GiB, by default) keep those tails few.
    Then k-NN with k = 32 over the same queries.  Reported: neighbours/s and the method's
    algorithmic bytes per second (cloud 12 B x N, centres 12 B x Q, offsets
    8 B x (Q + 1), indices 4 B x T) against the HBM peak."""
    import numpy as np
    import torch

    import cloudgen
    from paper_2502_11602_amd import GridIndex
    from paper_2502_11602_amd.autotune import pick_radius_schedule

    print("[bench] generating TLS scan: 20 M points", file=sys.stderr, flush=True)
    c = cloudgen.config2()
    xyz, qidx = c["xyz"], c["queries"]
    n, nq = len(xyz), len(qidx)
    dev = torch.device("cuda:0")
    x = torch.from_numpy(xyz).to(dev)
    q_in = torch.from_numpy(qidx).to(dev)
    budget = int(args.chunk_entries)
    E = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
    flavors = [f for f in args.tls_flavors.split(",") if f]
    out_fl = {}
    for fl in flavors:
        e0, e1, e2 = E(), E(), E()
        e0.record()
        gi = GridIndex(x, cell=0.25, flavor=fl)
        if args.radius_schedule != "auto":
            gi.set_radius_schedule(args.radius_schedule)
        e1.record()
        # the queries in the searches' processing order, so that every fill
        # range is spatially compact (rows then follow this order)
        q = q_in[gi.query_order(q_in).long()]
        e2.record()
        torch.cuda.synchronize()
        rec = {"build_ms": e0.elapsed_time(e1), "query_order_ms": e1.elapsed_time(e2),
               "radius": {}}

        def one_pass(r):
            ev = [E() for _ in range(3)]
            ev[0].record()
            off, _ = gi.radius_count(r, q, sync=False)
            ev[1].record()
            nch = 0
            for a, b, nbr in gi.radius_chunked(r, q, budget, offsets=off):
                nch += 1
            ev[2].record()
            torch.cuda.synchronize()
            return ev, int(off[-1]), nch

        for r in c["radii"]:
            if args.radius_schedule == "auto":
                # the radius schedule of this batch, by timing both count passes
                sched, sched_ms = pick_radius_schedule(gi, r, q)
            else:
                sched, sched_ms = args.radius_schedule, {}
            for _ in range(args.warmup):
                one_pass(r)
            cms, fms, tot, nch = [], [], 0, 0
            for _ in range(max(args.steps, 1)):
                ev, tot, nch = one_pass(r)
                cms.append(ev[0].elapsed_time(ev[1]))
                fms.append(ev[1].elapsed_time(ev[2]))
            cm, fm = float(np.median(cms)), float(np.median(fms))
            byt = 12 * n + 12 * nq + 8 * (nq + 1) + 4 * tot
            rec["radius"][str(r)] = {
                "schedule": sched, "schedule_count_ms": sched_ms,
                "count_ms": cm, "chunked_fill_ms": fm, "ranges": nch, "neighbours": tot,
                "mean_neighbours": tot / nq, "neighbours_per_s": tot / ((cm + fm) / 1e3),
                "queries_per_s": nq / ((cm + fm) / 1e3), "algorithmic_bytes": byt,
                "GB_per_s": byt / ((cm + fm) / 1e3) / 1e9,
                "hbm_frac": byt / ((cm + fm) / 1e3) / 1e9 / PEAK_HBM_GBS}
            print(f"[bench] tls {fl} r={r} ({sched}): {tot} neighbours in {nch} ranges, count {cm:.1f} ms,"
                  f" fill {fm:.1f} ms", file=sys.stderr, flush=True)
        k = c["k"]
        gi.knn(k, q)
        kms = []
        for _ in range(max(args.steps, 1)):
            a, b = E(), E()
            a.record()
            idx, d2 = gi.knn(k, q)
            b.record()
            torch.cuda.synchronize()
            kms.append(a.elapsed_time(b))
            del idx, d2
        rec["knn"] = {"k": k, "ms": float(np.median(kms)),
                      "queries_per_s": nq / (float(np.median(kms)) / 1e3)}
        print(f"[bench] tls {fl} knn k={k}: {rec['knn']['ms']:.1f} ms", file=sys.stderr, flush=True)
        out_fl[fl] = rec
        gi.close()
        del gi
        torch.cuda.empty_cache()
    # k-NN by voxel edge: near the scanner a 0.25 m voxel holds hundreds of
    # points, far more than 32 neighbours need (Section 5.3 sees k-NN suffer
    # on dense non-ALS clouds); the edge is chosen by timing, as the
    # autotuner does
    knn_cells = {}
    for cell in [float(v) for v in args.tls_knn_cells.split(",") if v]:
        gk = GridIndex(x, cell=cell, flavor=flavors[0])
        gk.knn(c["k"], q_in)
        kms = []
        for _ in range(max(args.steps, 1)):
            a, b = E(), E()
            a.record()
            idx, d2 = gk.knn(c["k"], q_in)
            b.record()
            torch.cuda.synchronize()
            kms.append(a.elapsed_time(b))
            del idx, d2
        knn_cells[str(cell)] = float(np.median(kms))
        gk.close()
        del gk
        torch.cuda.empty_cache()
        print(f"[bench] tls knn k={c['k']} at {cell} m voxels: {knn_cells[str(cell)]:.1f} ms",
              file=sys.stderr, flush=True)
    best = min(out_fl, key=lambda f: sum(v["count_ms"] + v["chunked_fill_ms"]
                                         for v in out_fl[f]["radius"].values()))
    rr = out_fl[best]["radius"]
    ms = sum(v["count_ms"] + v["chunked_fill_ms"] for v in rr.values())
    tot = sum(v["neighbours"] for v in rr.values())
    out = {"metric": "TLS radius search neighbours/s (count + range-by-range fill, "
                     "r = 0.1, 0.25, 0.5 m)",
           "value": tot / (ms / 1e3), "unit": "neighbours/s", "n_gpus": 1,
           "steps": max(args.steps, 1), "warmup": args.warmup, "ms_per_step": ms,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": f"TLS scan, {n} points, {nq} query points, 0.25 m voxels, "
                                  f"{best} map (best of {flavors}); fill ranges of at most "
                                  f"{budget} entries", "n_points": n, "n_queries": nq},
           "chunk_entries": budget, "flavors": out_fl,
           "knn_by_cell_ms": knn_cells}
    print(json.dumps(out), flush=True)


def _split(a, b):
    """Shares of queries where a visits fewer, more or as many voxels as b."""
    n = max(len(a), 1)
    return {"fewer": float((a < b).sum()) / n, "more": float((a > b).sum()) / n,
            "equal": float((a == b).sum()) / n}


def run_knnstats(args):
    """Density versus monotonic radius growth in k-NN (Section 3.5): on
    1 M uniform random points (cloudgen.uniform_cube: a 100 m cube, about one
    point per cubic metre) every point queries its k nearest, dense map, for
    voxel edges 0.5-4 m and k = 4-32.  The GPU runs the three schedules
    (rings, density growth, monotonic growth) and counts per query the
    voxels of its own taboo box under each growth schedule (Alg. 2 run for
    it alone, the paper's statistic: density growth fewer in 84.5 %, more in
    3.6 %, equal in 11.9 % of queries, on a cloud whose k and voxel edge it
    does not state) and of its wave's visited box (what the GPU scans), and
    times each schedule."""
    import numpy as np
    import torch

    import cloudgen
    from paper_2502_11602_amd import GridIndex

    xyz = cloudgen.uniform_cube()
    n = xyz.shape[0]
    dev = torch.device("cuda:0")
    x = torch.from_numpy(xyz).to(dev)
    E = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
    rows = []
    for cell in (0.5, 1.0, 2.0, 4.0):
        gi = GridIndex(x, cell=cell, flavor="dense")
        for k in (4, 8, 16, 32):
            rec = {"cell_m": cell, "k": k}
            own, wave, lists = {}, {}, {}
            for sched in ("rings", "density", "monotonic"):
                gi.set_knn_schedule(sched)
                gi.knn(k)
                torch.cuda.synchronize()
                ts = []
                for _ in range(max(args.steps, 1)):
                    a, b = E(), E()
                    a.record()
                    idx, d2 = gi.knn(k)
                    b.record()
                    torch.cuda.synchronize()
                    ts.append(a.elapsed_time(b))
                i2, e2, v = gi.knn_visited(k)
                v = v.cpu().numpy()
                own[sched], wave[sched] = v[:, 0], v[:, 1]
                lists[sched] = bool(torch.equal(idx, i2) and torch.equal(d2, e2))
                if sched != "rings":
                    lists[sched] = lists[sched] and bool(torch.equal(idx, ref_i)
                                                         and torch.equal(d2, ref_d))
                else:
                    ref_i, ref_d = idx, d2
                rec[f"{sched}_ms"] = float(np.median(ts))
                rec[f"{sched}_mean_wave_voxels"] = float(wave[sched].mean())
            rec["identical_lists"] = all(lists.values())
            rec["density_vs_monotonic_own"] = _split(own["density"], own["monotonic"])
            rec["mean_own_voxels"] = {"density": float(own["density"].mean()),
                                      "monotonic": float(own["monotonic"].mean())}
            rec["density_vs_rings_wave"] = _split(wave["density"], wave["rings"])
            rows.append(rec)
            print(f"[bench] knnstats s={cell} k={k}: density fewer "
                  f"{rec['density_vs_monotonic_own']['fewer']:.3f} more "
                  f"{rec['density_vs_monotonic_own']['more']:.3f}; rings {rec['rings_ms']:.2f} ms,"
                  f" density {rec['density_ms']:.2f} ms, monotonic {rec['monotonic_ms']:.2f} ms",
                  file=sys.stderr, flush=True)
        gi.close()
    gi = None
    ref = next(r for r in rows if r["cell_m"] == 1.0 and r["k"] == 16)
    best = min(ref["rings_ms"], ref["density_ms"], ref["monotonic_ms"])
    near = min(rows, key=lambda r: abs(r["density_vs_monotonic_own"]["fewer"] - 0.845)
               + abs(r["density_vs_monotonic_own"]["more"] - 0.036))
    out = {"metric": "k-NN queries/s, every point a query (uniform random cloud, k = 16)",
           "value": n / (best / 1e3), "unit": "queries/s", "n_gpus": 1,
           "steps": max(args.steps, 1), "warmup": 1, "ms_per_step": best,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": f"{n} uniform random points in a 100 m cube, dense map, "
                                  "voxel edges 0.5-4 m, k = 4-32 (value: 1 m voxels, k = 16)",
                      "n_points": n},
           "paper_density_vs_monotonic": {"fewer": 0.845, "more": 0.036, "equal": 0.119},
           "closest_row": {"cell_m": near["cell_m"], "k": near["k"],
                           **near["density_vs_monotonic_own"]},
           "rows": rows}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--radii", default="0.5,1,2,3")
    ap.add_argument("--ks", default="8,16,32")
    ap.add_argument("--flavor", default="dense")
    ap.add_argument("--cell", type=float, default=1.0)
    ap.add_argument("--points", type=int, default=10_000_000)
    ap.add_argument("--cpu-sample", type=int, default=20_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-flavor-compare", action="store_true")
    ap.add_argument("--no-kernel-compare", action="store_true")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run one device-to-device copy of this size before the steps "
                         "(a known-size kernel for scaling hardware byte counters)")
    ap.add_argument("--workload", default="als10m", choices=["als10m", "batched", "sweep", "agg", "knnstats", "tls"])
    ap.add_argument("--chunk-entries", type=int, default=1 << 35,
                    help="tls: neighbour entries per fill range (4 B each; the default "
                         "buffer is 128 GiB of the GPU's 288 GB)")
    ap.add_argument("--tls-flavors", default="sparse,mixed")
    ap.add_argument("--tls-knn-cells", default="0.1,0.25,0.5",
                    help="tls: voxel edges at which k-NN is also timed")
    ap.add_argument("--radius-schedule", default="auto", choices=["auto", "tiles", "groups"],
                    help="tls: the radius searches' work sharing")
    ap.add_argument("--agg-cell", type=float, default=0.5)
    ap.add_argument("--batch-scale", type=float, default=1.0)
    ap.add_argument("--batch-r", type=float, default=1.0)
    ap.add_argument("--batch-k", type=int, default=16)
    ap.add_argument("--tune-cache", default=None)
    ap.add_argument("--write-summary", action="store_true",
                    help="sweep: also write its profiles/ summary")
    ap.add_argument("--profile-summary", nargs=2, metavar=("STATS_DIR", "PMC_ROOT"),
                    help="write the profiles/ summaries from rocprofv3 output directories")
    ap.add_argument("--tls-profile-summary", nargs=2, metavar=("STATS_DIR", "BENCH_LOG"),
                    help="write the TLS workload's profiles/ summary")
    ap.add_argument("--agg-profile-summary", metavar="STATS_DIR",
                    help="write the aggregation workload's profiles/ summary")
    args = ap.parse_args()
    if args.profile_summary:
        profile_summary(*args.profile_summary)
        return
    if args.agg_profile_summary:
        agg_profile_summary(args.agg_profile_summary)
        return
    if args.tls_profile_summary:
        tls_profile_summary(*args.tls_profile_summary)
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(queries shard independently; see the design notes). Run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    if args.workload == "batched":
        run_batched(args)
        return
    if args.workload == "sweep":
        run_sweep(args)
        return
    if args.workload == "agg":
        run_agg(args)
        return
    if args.workload == "knnstats":
        run_knnstats(args)
        return
    if args.workload == "tls":
        run_tls(args)
        return

    import numpy as np
    import torch

    import cloudgen
    from paper_2502_11602_amd import GridIndex

    radii = [float(v) for v in args.radii.split(",") if v]
    ks = [int(v) for v in args.ks.split(",") if v]
    print(f"[bench] generating ALS tile: {args.points} points", file=sys.stderr, flush=True)
    cfg = cloudgen.config1(n=args.points)
    xyz = cfg["xyz"]
    n = xyz.shape[0]
    dev = torch.device("cuda:0")
    x = torch.from_numpy(xyz).to(dev)
    torch.cuda.synchronize()

    if args.copy_calibration_mib > 0:
        nel = args.copy_calibration_mib * (1 << 20) // 4
        src = torch.ones(nel, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"[bench] calibration copy: {nel * 4} bytes read, {nel * 4} bytes written",
              file=sys.stderr, flush=True)
        del src, dst

    E = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731

    def step(rec, flavor=args.flavor):
        ev = {"start": E()}
        ev["start"].record()
        ix = GridIndex(x, cell=args.cell, flavor=flavor)
        ev["build"] = E(); ev["build"].record()
        # (the build also plans the processing order of "every point" queries)
        totals = {}
        for r in radii:
            off, tot = ix.radius_count(r)
            ev[f"count{r}"] = E(); ev[f"count{r}"].record()
            nbr = ix.radius_fill(r, off, tot)
            ev[f"fill{r}"] = E(); ev[f"fill{r}"].record()
            totals[r] = tot
            del nbr, off
        for k in ks:
            idx, d2 = ix.knn(k)
            ev[f"knn{k}"] = E(); ev[f"knn{k}"].record()
            del idx, d2
        ix.close()
        if rec is not None:
            rec.append((ev, totals))

    for w in range(args.warmup):
        step(None)
        print(f"[bench] warmup {w + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    recs = []
    t0 = time.perf_counter()
    for s in range(args.steps):
        step(recs)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    print(f"[bench] {args.steps} timed steps in {wall:.3f} s", file=sys.stderr, flush=True)

    def avg(a, b):
        return sum(ev[a].elapsed_time(ev[b]) for ev, _ in recs) / len(recs)

    names = ["start", "build"]
    for r in radii:
        names += [f"count{r}", f"fill{r}"]
    names += [f"knn{k}" for k in ks]
    phase = {names[i]: avg(names[i - 1], names[i]) for i in range(1, len(names))}
    totals = recs[-1][1]
    ms_step = wall * 1e3 / args.steps
    nops = len(radii) + len(ks)
    value = nops * n / (ms_step / 1e3)

    radius = {}
    for r in radii:
        ms = phase[f"count{r}"] + phase[f"fill{r}"]
        radius[str(r)] = {"count_ms": phase[f"count{r}"], "fill_ms": phase[f"fill{r}"],
                          "queries_per_s": n / (ms / 1e3), "neighbours": totals[r],
                          "mean_neighbours": totals[r] / n}
    knn = {str(k): {"ms": phase[f"knn{k}"], "queries_per_s": n / (phase[f"knn{k}"] / 1e3)}
           for k in ks}

    # roofline of the dominant kernel: the radius fill at the largest radius
    # (it writes the CSR lists).  Algorithmic bytes per launch: query records
    # 16 B x Q + row offsets 8 B x Q + every stored point at least once 16 B x N
    # + neighbour indices 4 B x T.  Beside it, the whole search at that radius
    # (count + offsets + fill) against the method's own minimum: the FP32
    # cloud 12 B x N, the centres 12 B x Q, the offsets 8 B x (Q + 1) and the
    # indices 4 B x T.
    rdom = max(radii)
    T = totals[rdom]
    alg_bytes = 16 * n + 8 * n + 16 * n + 4 * T
    fill_s = phase[f"fill{rdom}"] / 1e3
    achieved = alg_bytes / fill_s / 1e9
    search_bytes = 12 * n + 12 * n + 8 * (n + 1) + 4 * T
    search_s = (phase[f"count{rdom}"] + phase[f"fill{rdom}"]) / 1e3
    roof = {"kernel": "radius fill", "radius_m": rdom, "bound": "hbm", "achieved": achieved,
            "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS,
            "traffic": counter_traffic(rdom),
            "algorithmic_bytes": alg_bytes, "launch_ms": phase[f"fill{rdom}"],
            "search": {"what": "count + offsets + fill", "algorithmic_bytes": search_bytes,
                       "ms": search_s * 1e3, "achieved": search_bytes / search_s / 1e9,
                       "frac": search_bytes / search_s / 1e9 / PEAK_HBM_GBS}}

    # the three voxel maps on the same step, one warm and one measured step
    # each, after the timed steps (config 1 compares the flavors)
    flavors = {}
    if not args.no_flavor_compare:
        for fl in ("dense", "sparse", "mixed"):
            step(None, fl)
            rec = []
            step(rec, fl)
            torch.cuda.synchronize()
            ev = rec[0][0]
            el = {names[i]: ev[names[i - 1]].elapsed_time(ev[names[i]]) for i in range(1, len(names))}
            flavors[fl] = {"build_ms": el["build"],
                           "radius_ms": {str(r): el[f"count{r}"] + el[f"fill{r}"] for r in radii},
                           "knn_ms": {str(k): el[f"knn{k}"] for k in ks}}
            print(f"[bench] flavor {fl} done", file=sys.stderr, flush=True)

    # the cube and cylinder kernels of Alg. 1 on the same tile (outside the
    # timed steps): count + fill per radius, one warm and one measured pass
    shapes = {}
    if not args.no_kernel_compare:
        ix = GridIndex(x, cell=args.cell, flavor=args.flavor)
        # Alg. 2's density-growth schedule for k-NN (same lists as the rings)
        ix.set_knn_schedule("density")
        shapes["knn_density_schedule"] = {}
        for k in ks:
            for rep in range(2):
                a, b = E(), E()
                a.record()
                idx, d2 = ix.knn(k)
                b.record()
                torch.cuda.synchronize()
            shapes["knn_density_schedule"][str(k)] = {"ms": a.elapsed_time(b)}
            del idx, d2
        ix.set_knn_schedule("rings")
        for kern in ("cube", "cylinder"):
            shapes[kern] = {}
            for r in radii:
                for rep in range(2):
                    a, b = E(), E()
                    a.record()
                    off, nbr = ix.radius(r, kernel=kern)
                    b.record()
                    torch.cuda.synchronize()
                shapes[kern][str(r)] = {"ms": a.elapsed_time(b), "neighbours": int(nbr.numel())}
                del off, nbr
        ix.close()
        print("[bench] cube / cylinder done", file=sys.stderr, flush=True)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": (f"ALS tile, {n} points over 1 km x 1 km (terrain, buildings, "
                         "multi-return vegetation), every point a query; build "
                         f"({args.flavor}, {args.cell} m voxels) + radius search r in "
                         f"{radii} m + k-NN k in {ks}"),
            "n_points": n, "queries_per_batch": n, "radii_m": radii, "ks": ks,
            "flavor": args.flavor, "cell_m": args.cell,
        },
        "build_ms": phase["build"],
        "build_mpts_s": n / (phase["build"] / 1e3) / 1e6,
        "radius": radius,
        "knn": knn,
        "roofline": roof,
        "flavors": flavors,
        "kernels": shapes,
    }
    if not args.no_cpu_baseline:
        nth = len(os.sched_getaffinity(0))
        print(f"[bench] cpu baseline: oracle on {nth} threads", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(xyz, radii, ks, args.cell, args.cpu_sample, nth)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
