"""Benchmark: componentwise PageRank vs plain power series on one MI355X.

One step = one pr_solve of the componentwise method (Sec. 4.3: boundary
mass, one-vertex components, CAC sweeps, SCC power series from P_0 = W'_C
stopped on the certified geometric tail estimate, output, and the FP64
residual certificate of Sec. 4.4) on the web-like graph of 1M vertices / 10M
edges, with the plan resident on the device.  Timed the same way beside it,
each leg right after two untimed solves of its own: the plain whole-graph
power series (Sec. 5.2, method 1) with the same stop rule (the like-for-like
comparison) and with the plain 1-norm stop, the componentwise solve with the
plain stop, with the learned starting guess (both stop rules), with small
SCCs solved directly, and cold (a fresh W every step and every gang launched
for the worst-case term bound).  All are certified to 1e-6.

Prints ONE JSON line.  --gpus N > 1 is refused (single-GPU build).
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

METRIC = "GEdge-iter/s + time to 1e-6 rel err: componentwise(+warm start) vs plain PR"
HBM_PEAK_GBS = 8000.0

# Algorithmic bytes per unit of work (int32 indices, FP32 or FP64 terms, FP64 R):
#  term edge  4 B source index + one term gather (4 B mixed, 8 B FP64)
#  term row   row pointer 4 + 1/outdeg 4 + term write (4 | 8) + R read and write 16
#  once edge  4 B source index + 8 B x gather (boundary and CAC edges, and the
#             one compulsory load of an LDS-resident SCC's edges)
#  once row   W 8 + perm 4 + two row pointers 8 + R out 8 + x 8 + 1/outdeg 8
B_TERM_EDGE = {0: 8, 1: 12}
B_TERM_ROW = {0: 28, 1: 32}
B_ONCE_EDGE = 12
B_ONCE_ROW = 44
FAMILIES = ["k_segment", "k_gang", "k_gang_hubs", "k_reduce"]


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def family_bytes(fam, info, st, prec, plain):
    """Algorithmic bytes moved by all launches of one kernel family in one solve."""
    if fam == 0:  # segments: every row and edge outside the gangs once
        rows = info["n"] - info["v_gang"]
        edges = info["m"] - info["m_gang_internal"] - info["m_gang_between"]
        return rows * B_ONCE_ROW + edges * B_ONCE_EDGE
    if fam == 1:  # gang terms
        if plain:
            terms = st["iters_max"] + 1
            return terms * (info["m"] * B_TERM_EDGE[prec] + info["n"] * B_TERM_ROW[prec]) + info["n"] * B_ONCE_ROW
        gang_term_edges = st["gang_edge_iters"]
        gang_term_rows = st["gang_vert_iters"]
        return (gang_term_edges * B_TERM_EDGE[prec] + gang_term_rows * B_TERM_ROW[prec]
                + info["v_gang"] * B_ONCE_ROW + info["m_gang_between"] * B_ONCE_EDGE)
    return 0


def roofline(fam, info, st, prec, plain, traffic):
    cnt = st["kt_count"][fam]
    ms = st["kt_ms"][fam]
    b = family_bytes(fam, info, st, prec, plain)
    per_launch = b / max(cnt, 1)
    avg_ms = ms / max(cnt, 1)
    ach = per_launch / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    out = {"bound": "hbm", "achieved": round(ach, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic,
           "kernel": FAMILIES[fam], "launches_per_solve": cnt, "avg_launch_us": round(avg_ms * 1e3, 3),
           "alg_bytes_per_launch": int(per_launch)}
    if traffic and avg_ms > 0:
        # the counted memory-side bytes over the same duration: how close the
        # kernel runs to the bandwidth limit in the bytes it actually moves
        out["traffic_gbs"] = round(traffic / (avg_ms * 1e-3) / 1e9, 2)
        out["traffic_frac"] = round(out["traffic_gbs"] / HBM_PEAK_GBS, 4)
    return out


def load_traffic(path, kernel, shape=None):
    """HBM bytes per launch of `kernel` ("family/method") from a committed
    counter summary, or None when there is none, the kernel sources changed
    since the counters were taken, or they were taken at another launch shape
    (rows per wavefront, small cutoff, team edges) than `shape`."""
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("source_hash") != source_hash() or kernel not in d.get("kernels", {}):
        return None
    k = d["kernels"][kernel]
    if shape is not None and k.get("shape") != shape:
        return None
    return k["hbm_bytes_per_launch"]


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _strip_comments(src):
    """C/C++ source without comments and blank runs: what the compiler sees."""
    import re

    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
    src = re.sub(r"//[^\n]*", "", src)
    return re.sub(r"\s+", " ", src).strip()


def source_hash(read=None):
    """Hash of the library's sources with comments removed: a counter summary
    stays valid across comment-only edits and is void after any code change."""
    import hashlib

    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1609_09068_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".h", ".cpp")):
            if read is None:
                with open(os.path.join(csrc, name)) as f:
                    text = f.read()
            else:
                text = read(name)
            h.update(name.encode() + _strip_comments(text).encode())
    return h.hexdigest()[:16]


def summarize_pmc(fetch_dir, write_dir, calib_mb, out, method, shape=None):
    """Turn two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE; KiB per
    dispatch) into bytes per launch per kernel family, scaled by what the
    same counters read for a plain device copy of calib_mb MiB."""
    import csv
    import glob

    def read(d, counter):
        rows = []
        for fn in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            with open(fn) as f:
                for r in csv.DictReader(f):
                    if r.get("Counter_Name") == counter:
                        rows.append((r["Kernel_Name"], float(r["Counter_Value"])))
        return rows

    res = {}
    calib = {}
    for counter, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        rows = read(d, counter)
        copy = [v for k, v in rows if "elementwise" in k.lower() or "copy" in k.lower()]
        copy = [v for v in copy if v > 0.5 * calib_mb * 1024]
        if not copy:
            raise SystemExit(f"no calibration copy dispatch found for {counter}")
        factor = calib_mb * 1024.0 / float(np.median(copy))
        calib[counter] = {"copy_mib": calib_mb, "counter_kib_median": float(np.median(copy)), "factor": factor}
        for fam in FAMILIES:
            vals = [v for k, v in rows if (fam + "<") in k or (fam + "_w3<") in k or k.endswith(fam) or (fam + "(") in k]
            if fam == "k_gang":
                vals = [v for k, v in rows if "k_gang<" in k]
            if vals:
                res.setdefault(fam, {})[counter] = {"dispatches": len(vals), "kib_mean": float(np.mean(vals)),
                                                    "bytes_per_launch": float(np.mean(vals)) * 1024 * factor}
    kern = {}
    for fam, d in res.items():
        if "FETCH_SIZE" in d and "WRITE_SIZE" in d:
            r = d["FETCH_SIZE"]["bytes_per_launch"]
            w = d["WRITE_SIZE"]["bytes_per_launch"]
            kern[fam] = {"read_bytes_per_launch": int(r), "write_bytes_per_launch": int(w),
                         "hbm_bytes_per_launch": int(r + w), "dispatches": d["FETCH_SIZE"]["dispatches"],
                         "shape": shape}
    doc = {}
    if os.path.exists(out):
        with open(out) as f:
            doc = json.load(f)
        if doc.get("source_hash") != source_hash():
            doc = {}
    doc["source_hash"] = source_hash()
    doc.setdefault("calibration", {})[method] = calib
    for fam, v in kern.items():
        doc.setdefault("kernels", {})[f"{fam}/{method}"] = v
    with open(out, "w") as f:
        json.dump(doc, f, indent=1)
    print(json.dumps(doc))


def calib_copy(torch, mib):
    """A plain device copy of known size: what FETCH_SIZE / WRITE_SIZE read for it
    scales the kernel's counters to bytes."""
    nb = mib * (1 << 20) // 4
    a = torch.ones(nb, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    log(f"calibration copy: {mib} MiB read + {mib} MiB write")


def residual_bound(g, c, R, AT=None):
    from oracle.pagerank import residual_bound as rb

    return rb(g.n, g.row_ptr, g.col, c, np.ones(g.n), R, AT)


def run_study(args, pr, torch, g, lv, info, W, R, t_part, t_build):
    rows = []
    AT = None
    for c in (0.85, 0.99):
        for prec in (0, 1):
            for meth, tail in ((0, 0), (0, 1), (1, 0)):
                name = (("componentwise" + ("+tail_estimate" if tail else "")) if meth == 0 else "plain") + \
                       ("/mixed" if prec == 0 else "/fp64")
                st = None
                ms = []
                for rep in range(1 + max(args.steps, 1)):
                    rc, st = pr.pr_solve(lv, c, W, R, method=meth, precision=prec, eps=args.eps, kernel_timing=1,
                                         tail_estimate=tail)
                    if rep:
                        ms.append(st["kernel_ms"])
                bound, AT = residual_bound(g, c, R.cpu().numpy(), AT)
                t = float(np.median(ms))
                kt = st["kt_ms"]
                fam = 1 if meth == 1 else int(np.argmax(kt))
                b = family_bytes(fam, info, st, prec, meth == 1)
                row = {"c": c, "path": name, "ms": round(t, 3), "gedge_iter_s": round(st["edge_iters"] / t / 1e6, 3),
                       "terms_max": st["iters_max"], "edge_iters": st["edge_iters"],
                       "rel_l1_bound_vs_oracle_residual": bound, "cert_rel": st["cert_rel"],
                       "dominant_kernel": FAMILIES[fam],
                       "dominant_kernel_alg_gbs": round(b / (kt[fam] * 1e-3) / 1e9, 1) if kt[fam] > 0 else None}
                log(json.dumps(row))
                rows.append(row)
    print(json.dumps({"study": "precision", "config": args.config, "n": g.n, "m": g.m, "eps": args.eps,
                      "partition_ms": round(t_part * 1e3, 1), "build_ms": round(t_build * 1e3, 1),
                      "rows": rows, "device": torch.cuda.get_device_name(0)}), flush=True)


def run_tol_sweep(args, pr, torch, g, lv, info, W, R, t_part, t_build):
    """Time to solve against the tolerance (the experiment of Sec. 5.2 and
    the B-A figure): componentwise and plain at eps 1e-2 ... 1e-10, hipGraph
    replays, with each result's error bound from the oracle's FP64 residual."""
    rows = []
    AT = None
    for eps in (1e-2, 1e-4, 1e-6, 1e-8, 1e-10):
        for meth, direct, tail in ((0, 0, 0), (0, 24, 0), (0, 0, 1), (1, 0, 0)):
            prec = 0 if eps >= 1e-6 else 1  # FP32 terms cannot certify below about 1e-7
            for _ in range(2):
                pr.pr_solve(lv, args.c, W, R, method=meth, precision=prec, eps=eps, use_graph=1, small_direct=direct,
                            tail_estimate=tail)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                rc, st = pr.pr_solve(lv, args.c, W, R, method=meth, precision=prec, eps=eps, use_graph=1,
                                     small_direct=direct, tail_estimate=tail)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) / args.steps * 1e3
            bound, AT = residual_bound(g, args.c, R.cpu().numpy(), AT)
            name = "plain" if meth == 1 else ("componentwise" + ("+small_direct" if direct else "")
                                              + ("+tail_estimate" if tail else ""))
            row = {"eps": eps, "method": name,
                   "precision": "mixed" if prec == 0 else "fp64", "ms": round(ms, 3),
                   "terms_max": st["iters_max"], "edge_iters": st["edge_iters"], "cert_rel": st["cert_rel"],
                   "rel_l1_bound_vs_oracle_residual": bound}
            log(json.dumps(row))
            rows.append(row)
    print(json.dumps({"study": "tolerance", "config": args.config, "n": g.n, "m": g.m,
                      "levels": info["n_levels"], "scc_vertices": info["v_scc"],
                      "partition_ms": round(t_part * 1e3, 1), "build_ms": round(t_build * 1e3, 1),
                      "rows": rows, "device": torch.cuda.get_device_name(0)}), flush=True)


def run_c4(args, pr, torch):
    """The learned-start evaluation: fresh graphs of the 1M-vertex web-like
    recipe (seeds 4901-4905, never seen in training), time and terms to 1e-6
    with and without the guess, under both stop rules, and the guess's
    fallback rate per component (gang SCCs only, and every SCC)."""
    from graphgen import config_graph

    net = pr.Mlp.load_file(args.warm_net)
    rows = []
    for seed in range(4901, 4906):
        g = config_graph("c2_web_1m", seed=seed)
        part = pr.pr_partition(g.row_ptr, g.col)
        bo = dict(rows_per_wave=args.rows_per_wave or 64, small_cutoff=args.small_cutoff or 16,
                  team_edges=args.team_edges or 16384)
        lv = pr.pr_build_levels(part, g.row_ptr, g.col, **bo)
        W = torch.ones(g.n, dtype=torch.float64, device="cuda")
        R = torch.empty_like(W)
        row = {"seed": seed, "n": g.n, "m": g.m, "gang_vertices": lv.info()["v_gang"]}
        for name, extra in (("uniform_start", {}), ("guess", dict(warm_start=net)),
                            ("uniform_start_tail", dict(tail_estimate=1)),
                            ("guess_tail", dict(warm_start=net, tail_estimate=1)),
                            ("guess_every_scc", dict(warm_start=net, warm_scope=1))):
            for _ in range(2):
                pr.pr_solve(lv, args.c, W, R, eps=args.eps, use_graph=1, **extra)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                rc, st = pr.pr_solve(lv, args.c, W, R, eps=args.eps, use_graph=1, **extra)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) / args.steps * 1e3
            d = {"ms": round(ms, 4), "terms_sum": st["iters_sum"], "terms_max": st["iters_max"],
                 "edge_iters": st["edge_iters"], "cert_rel": st["cert_rel"]}
            if "warm_start" in extra:
                tot = st["ws_accepted"] + st["ws_rejected"]
                d.update(kept=st["ws_accepted"], fell_back=st["ws_rejected"],
                         fallback_rate_per_component=round(st["ws_rejected"] / max(tot, 1), 4))
            row[name] = d
        log(json.dumps(row))
        rows.append(row)
        lv.free()
        part.free()

    def mean(key, leg):
        return round(float(np.mean([r[leg][key] for r in rows])), 4)

    summary = {leg: {"ms": mean("ms", leg), "terms_sum": mean("terms_sum", leg), "terms_max": mean("terms_max", leg)}
               for leg in ("uniform_start", "guess", "uniform_start_tail", "guess_tail", "guess_every_scc")}
    print(json.dumps({"study": "learned start (fresh 1M-vertex web-like graphs)", "eps": args.eps, "c": args.c,
                      "network": os.path.relpath(args.warm_net, ROOT), "rows": rows, "mean": summary,
                      "device": torch.cuda.get_device_name(0)}), flush=True)


def run_weighted(args, pr, torch):
    """Weighted graphs (Def. 3.4): the workload's graph with seeded synthetic
    transition weights, uniform in [0.5, 1.5), on a weighted plan; time to
    eps for the componentwise and plain series under both stop rules, the
    same graph unweighted for the cost of the weights.  Accuracy is the
    solves' own FP64 residual certificate (parity with the oracle is in the
    tests)."""
    from graphgen import config_graph

    g = config_graph(args.config)
    w = np.random.default_rng(7001).uniform(0.5, 1.5, g.m)
    part = pr.pr_partition(g.row_ptr, g.col)
    bo = dict(rows_per_wave=args.rows_per_wave or 64, small_cutoff=args.small_cutoff or 16,
              team_edges=args.team_edges or 16384)
    lvw = pr.pr_build_levels(part, g.row_ptr, g.col, weight=w, **bo)
    lvu = pr.pr_build_levels(part, g.row_ptr, g.col, **bo)
    W = torch.ones(g.n, dtype=torch.float64, device="cuda")
    R = torch.empty_like(W)
    out = {"study": "weighted graph (synthetic transition weights, uniform [0.5, 1.5))", "config": args.config,
           "n": g.n, "m": g.m, "c": args.c, "eps": args.eps, "shape": bo, "legs": {},
           "device": torch.cuda.get_device_name(0)}
    legs = (("weighted_componentwise_tail", lvw, dict(tail_estimate=1)),
            ("weighted_componentwise_plain_stop", lvw, {}),
            ("weighted_plain_tail", lvw, dict(method=1, tail_estimate=1)),
            ("weighted_plain_plain_stop", lvw, dict(method=1)),
            ("unweighted_componentwise_tail", lvu, dict(tail_estimate=1)),
            ("unweighted_plain_tail", lvu, dict(method=1, tail_estimate=1)))
    for name, lv, extra in legs:
        for _ in range(max(args.warmup, 2)):
            pr.pr_solve(lv, args.c, W, R, eps=args.eps, use_graph=1, **extra)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            rc, st = pr.pr_solve(lv, args.c, W, R, eps=args.eps, use_graph=1, **extra)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / args.steps * 1e3
        d = {"ms": round(ms, 4), "terms_sum": st["iters_sum"], "terms_max": st["iters_max"],
             "edge_iters": st["edge_iters"], "gedge_iter_s": round(st["edge_iters"] / (ms * 1e-3) / 1e9, 3),
             "cert_rel": st["cert_rel"], "refine_rounds": st["refine_rounds"], "rc": rc}
        out["legs"][name] = d
        log(name, json.dumps(d))
    L = out["legs"]
    out["speedup_vs_plain_tail"] = round(L["weighted_plain_tail"]["ms"] / L["weighted_componentwise_tail"]["ms"], 3)
    out["speedup_vs_plain_both_plain_stop"] = round(
        L["weighted_plain_plain_stop"]["ms"] / L["weighted_componentwise_plain_stop"]["ms"], 3)
    out["weighted_over_unweighted_componentwise"] = round(
        L["weighted_componentwise_tail"]["ms"] / L["unweighted_componentwise_tail"]["ms"], 3)
    print(json.dumps(out), flush=True)
    lvw.free()
    lvu.free()
    part.free()


def run_stream_probe(args, pr, torch):
    """Achievable read bandwidth (pr_bandwidth_probe): buffers far larger than
    the 256 MB MALL (HBM-bound), ones that stay resident in it (after the
    untimed passes each pass reads from the MALL), and one that fits an XCD's
    4 MB L2.  The gather kernels' rooflines are read against these."""
    out = {"study": "stream probe", "device": torch.cuda.get_device_name(0), "kernel": "pr_bandwidth_probe", "rows": []}
    for label, mib, reps in (("hbm", 4096, 10), ("hbm", 2048, 20), ("mall", 200, 100), ("mall", 96, 200),
                             ("mall", 40, 400), ("l2", 2, 2000)):
        x = torch.ones(mib * (1 << 20) // 4, dtype=torch.float32, device="cuda")
        ms = pr.bandwidth_probe(x, reps)
        row = {"what": f"read {mib} MiB ({label})", "ms": round(ms, 5),
               "gb_s": round(mib * (1 << 20) / (ms * 1e-3) / 1e9, 1)}
        out["rows"].append(row)
        log(json.dumps(row))
        del x
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="c2_web_1m")
    ap.add_argument("--c", type=float, default=0.85)
    ap.add_argument("--eps", type=float, default=1e-6)
    ap.add_argument("--precision", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--no-check", action="store_true", help="skip the accuracy check against the oracle")
    ap.add_argument("--check", choices=["auto", "reference", "residual"], default="auto",
                    help="accuracy against the oracle: its FP64 series at eps 1e-12 (reference), or the bound "
                         "||W - (I - cA^T)R||_1 / ((1-c)||R||_1) from one FP64 product (residual); auto picks the "
                         "reference up to 20M edges")
    ap.add_argument("--study", action="store_true",
                    help="precision study: c in {0.85, 0.99} x {mixed, fp64} x {componentwise, plain}; prints one "
                         "JSON line of its own instead of the benchmark line")
    ap.add_argument("--stream-probe", action="store_true",
                    help="achievable HBM / MALL / L2 read bandwidth of the device; prints one JSON line of its own")
    ap.add_argument("--weighted", action="store_true",
                    help="weighted-graph study: the workload with synthetic transition weights (one JSON line)")
    ap.add_argument("--c4", action="store_true",
                    help="learned-start evaluation on five fresh 1M-vertex web-like graphs; prints one JSON line "
                         "of its own instead of the benchmark line")
    ap.add_argument("--tol-sweep", action="store_true",
                    help="time against the tolerance (eps 1e-2 ... 1e-10), componentwise and plain; prints one "
                         "JSON line of its own instead of the benchmark line")
    ap.add_argument("--graph", type=int, default=1,
                    help="time hipGraph replays of the solve (1, default) or eager launches (0); the per-kernel "
                         "durations always come from a second, eager pass with an event pair around every launch")
    ap.add_argument("--rows-per-wave", type=int, default=0)
    ap.add_argument("--small-cutoff", type=int, default=0)
    ap.add_argument("--team-edges", type=int, default=0)
    ap.add_argument("--seg-waves", type=int, default=0, choices=[0, 2, 3],
                    help="workgroups per CU of the tail-estimate segment kernel (0: default or autotuned)")
    ap.add_argument("--autotune", type=int, default=1, choices=[0, 1, 2],
                    help="plan autotuner: 0 off, 1 cached or sweep, 2 sweep")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="also run a plain device copy of this size (HBM counter calibration)")
    ap.add_argument("--traffic", default=None,
                    help="committed counter summary that supplies roofline.traffic "
                         "(default: profiles/hbm_traffic_<config>.json)")
    ap.add_argument("--no-warm", action="store_true", help="no starting guess in the headline step")
    ap.add_argument("--tail-estimate", type=int, default=1, choices=[0, 1],
                    help="headline step stops each SCC series on the certified geometric tail estimate")
    ap.add_argument("--warm-net", default=os.path.join(ROOT, "paper_1609_09068_amd", "data", "warm_web.prmlp"))
    ap.add_argument("--only", choices=["componentwise", "plain"],
                    help="run one method only (counter runs: one kernel family per method)")
    ap.add_argument("--summarize-pmc", nargs=3, metavar=("FETCH_DIR", "WRITE_DIR", "OUT"),
                    help="write a counter summary from two rocprofv3 --pmc runs and exit "
                         "(with --only: the method those runs used)")
    args = ap.parse_args()
    if args.summarize_pmc:
        shape = None
        if args.rows_per_wave and args.small_cutoff and args.team_edges:
            shape = {"rows_per_wave": args.rows_per_wave, "small_cutoff": args.small_cutoff,
                     "team_edges": args.team_edges, "seg_waves": args.seg_waves or 2}
        summarize_pmc(args.summarize_pmc[0], args.summarize_pmc[1], args.calib_copy_mb or 1024,
                      args.summarize_pmc[2], args.only or "componentwise", shape)
        return
    if args.traffic is None:
        args.traffic = os.path.join(ROOT, "profiles", f"hbm_traffic_{args.config}.json")
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU only; --gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1609_09068_amd as pr
    from graphgen import config_graph

    torch.cuda.set_device(0)
    if args.stream_probe:
        run_stream_probe(args, pr, torch)
        return
    if args.c4:
        run_c4(args, pr, torch)
        return
    if args.weighted:
        run_weighted(args, pr, torch)
        return
    dev_name = torch.cuda.get_device_name(0)
    log("device", dev_name)
    t0 = time.perf_counter()
    g = config_graph(args.config, log=log)
    log(f"graph {args.config}: n={g.n} m={g.m} gen {time.perf_counter() - t0:.1f}s")

    t0 = time.perf_counter()
    part = pr.pr_partition(g.row_ptr, g.col)
    t_part = time.perf_counter() - t0
    log(f"partition {t_part * 1e3:.1f} ms: comps={part.n_comp} levels={part.n_levels}")
    bopts = {}
    if args.rows_per_wave:
        bopts["rows_per_wave"] = args.rows_per_wave
    if args.small_cutoff:
        bopts["small_cutoff"] = args.small_cutoff
    if args.team_edges:
        bopts["team_edges"] = args.team_edges
    if args.seg_waves:
        bopts["seg_waves"] = args.seg_waves
    if args.autotune and not (args.rows_per_wave or args.small_cutoff or args.team_edges or args.seg_waves):
        bopts["autotune"] = args.autotune
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lv = pr.pr_build_levels(part, g.row_ptr, g.col, **bopts)
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t0
    info = lv.info()
    log(f"build {t_build * 1e3:.1f} ms: {info}")

    W = torch.ones(g.n, dtype=torch.float64, device="cuda")
    R = torch.empty_like(W)
    Rp = torch.empty_like(W)
    if args.study:
        run_study(args, pr, torch, g, lv, info, W, R, t_part, t_build)
        return
    if args.tol_sweep:
        run_tol_sweep(args, pr, torch, g, lv, info, W, R, t_part, t_build)
        return
    common = dict(eps=args.eps, precision=args.precision, use_graph=args.graph, kernel_timing=0)

    def run(method, Rout, steps, **extra):
        stats = []
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            rc, st = pr.pr_solve(lv, args.c, W, Rout, method=method, **{**common, **extra})
            stats.append(st)
        torch.cuda.synchronize()
        return (time.perf_counter() - t), stats

    if args.only:
        # counter runs: a few solves of one method, then the calibration copy
        # the legs the rooflines use: the headline (componentwise with the
        # tail-estimate stop) and the plain series with the plain stop
        meth = 0 if args.only == "componentwise" else 1
        for _ in range(args.warmup + args.steps):  # eager launches: one profiler record per kernel
            run(meth, R, 1, use_graph=0, **(dict(tail_estimate=args.tail_estimate) if meth == 0 else {}))
        if args.calib_copy_mb:
            calib_copy(torch, args.calib_copy_mb)
        log(f"{args.only}: {args.warmup + args.steps} solves done")
        return
    net = None
    if not args.no_warm:
        if not os.path.exists(args.warm_net):
            raise SystemExit(f"bench.py: trained network {args.warm_net} missing (use --no-warm)")
        net = pr.Mlp.load_file(args.warm_net)
    tail = dict(tail_estimate=args.tail_estimate)
    # the legs, each timed as `steps` solves right after two untimed ones (so
    # a leg never pays another leg's graph capture or gang budget)
    legs = [("componentwise", 0, dict(tail))]  # the headline step
    if net is not None:
        legs += [("componentwise_guess", 0, dict(tail, warm_start=net)),
                 ("componentwise_guess_plain_stop", 0, dict(warm_start=net))]
    legs += [("componentwise_plain_stop", 0, {}),
             ("componentwise_gauss_seidel4", 0, dict(gs_blocks=4)),
             ("componentwise_small_direct", 0, dict(small_direct=24)),
             ("plain", 1, dict(tail)),
             ("plain_plain_stop", 1, {})]
    res = {}
    for _ in range(args.warmup):
        for name, meth, extra in legs:
            run(meth, R, 1, **extra)
    mode = "hipGraph replay" if args.graph else "eager launches"
    log(f"warmup done; timing {args.steps} solves of each leg ({mode})")
    for name, meth, extra in legs:
        Rl = torch.empty_like(W)
        run(meth, Rl, 2, **extra)
        t, sts = run(meth, Rl, args.steps, **extra)
        res[name] = (t / args.steps * 1e3, sts[-1], Rl)
        log(f"{name}: {res[name][0]:.3f} ms/step")
    # cold: a different weight vector every step (resident before the timed
    # region) and every gang launched for the worst-case term bound
    gen = torch.Generator(device="cuda")
    gen.manual_seed(12345)
    Wc = [torch.rand(g.n, dtype=torch.float64, device="cuda", generator=gen) + 0.5 for _ in range(args.steps + 2)]
    Rc = torch.empty_like(W)
    for q in range(2):
        pr.pr_solve(lv, args.c, Wc[q], Rc, method=0, cold=1, **{**common, **tail})
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for q in range(args.steps):
        rc, st_cold = pr.pr_solve(lv, args.c, Wc[q + 2], Rc, method=0, cold=1, **{**common, **tail})
    torch.cuda.synchronize()
    ms_cold = (time.perf_counter() - t0) / args.steps * 1e3
    log(f"componentwise, cold (fresh W each step, worst-case gang budget): {ms_cold:.3f} ms/step")
    # per-kernel durations: the same solves, eager, an event pair around every
    # launch on the solve stream (the events add a little host time per launch)
    t_ecw, st_ecw = run(0, R, args.steps, use_graph=0, kernel_timing=1, **tail)
    t_epl, st_epl = run(1, Rp, args.steps, use_graph=0, kernel_timing=1)
    log(f"eager with launch events: componentwise {t_ecw / args.steps * 1e3:.3f} ms/step, "
        f"plain {t_epl / args.steps * 1e3:.3f} ms/step")

    if args.calib_copy_mb:
        calib_copy(torch, args.calib_copy_mb)

    ms_cw, s, _ = res["componentwise"]
    ms_pl, sp, _ = res["plain"]
    ms_pl_nt, sp_nt, _ = res["plain_plain_stop"]
    ms_cw_nt = res["componentwise_plain_stop"][0]

    def mean_stats(sts):
        d = dict(sts[-1])
        d["kt_ms"] = list(np.mean([x["kt_ms"] for x in sts], axis=0))
        d["kernel_ms"] = float(np.mean([x["kernel_ms"] for x in sts]))
        return d

    mcw = mean_stats(st_ecw)
    mpl = mean_stats(st_epl)
    value = s["edge_iters"] / (ms_cw * 1e-3) / 1e9
    dom = int(np.argmax(mcw["kt_ms"])) if any(mcw["kt_ms"]) else 0
    shape = {k: info[k] for k in ("rows_per_wave", "small_cutoff", "team_edges", "seg_waves")}
    traffic_cw = load_traffic(args.traffic, FAMILIES[dom] + "/componentwise", shape)
    roof = roofline(dom, info, mcw, args.precision, False, traffic_cw)
    roof_spmv = roofline(1, info, mpl, args.precision, True, load_traffic(args.traffic, "k_gang/plain", shape))
    roof_spmv["what"] = "plain whole-graph power series, one launch per term (the SpMV phase)"
    kt = {"componentwise": {FAMILIES[i]: {"ms": round(mcw["kt_ms"][i], 4), "launches": mcw["kt_count"][i]}
                            for i in range(4)},
          "plain_plain_stop": {FAMILIES[i]: {"ms": round(mpl["kt_ms"][i], 4), "launches": mpl["kt_count"][i]}
                               for i in range(4)}}

    acc = None
    check = args.check if args.check != "auto" else ("reference" if g.m <= 20_000_000 else "residual")
    if not args.no_check and check == "reference":
        from oracle.pagerank import pagerank_power_series

        t0 = time.perf_counter()
        ref, kref, _ = pagerank_power_series(g.n, g.row_ptr, g.col, args.c, np.ones(g.n), eps=1e-12)
        log(f"oracle reference (eps 1e-12, {kref} iterations) {time.perf_counter() - t0:.1f}s")
        acc = {name: float(np.abs(Rl.cpu().numpy() - ref).sum() / ref.sum()) for name, (_, _, Rl) in res.items()}
        acc["reference"] = f"oracle plain power series, FP64, eps 1e-12 ({kref} terms)"
    elif not args.no_check:
        AT = None
        acc = {}
        for name, (_, _, Rl) in res.items():
            acc[name], AT = residual_bound(g, args.c, Rl.cpu().numpy(), AT)
        acc["reference"] = "bound from the oracle's FP64 residual ||W - (I - cA^T)R||_1 / ((1-c)||R||_1)"
    if acc is not None:
        acc["cert_rel"] = {name: st["cert_rel"] for name, (_, st, _) in res.items()}
        if not args.no_check:
            from oracle.pagerank import residual_bound as rb

            acc["componentwise_cold_last_step"] = rb(g.n, g.row_ptr, g.col, args.c, Wc[args.steps + 1].cpu().numpy(),
                                                     Rc.cpu().numpy())[0]

    cpu = None
    if not args.no_cpu:
        from threadpoolctl import threadpool_limits

        from oracle.componentwise import componentwise_solve

        with threadpool_limits(limits=1):
            t0 = time.perf_counter()
            Ro, sto = componentwise_solve(g.n, g.row_ptr, g.col, args.c, np.ones(g.n), eps=args.eps,
                                          return_stats=True, tail=bool(args.tail_estimate))
            t_or = time.perf_counter() - t0
        part_d = part.as_dict()
        scc = part_d["comp_type"] == 1
        e_int = np.zeros(part.n_comp)
        src = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
        keep = (src != g.col) & (part_d["comp"][src] == part_d["comp"][g.col])
        np.add.at(e_int, part_d["comp"][src[keep]], 1)
        e_iter_or = float(np.sum(sto["iters"][scc] * e_int[scc])) + (info["m_between"] + info["m_cac_internal"])
        cpu = {"value": round(e_iter_or / t_or / 1e9, 5), "unit": "GEdge-iter/s", "cores": 1, "kind": "oracle",
               "sample": f"the whole {args.config} solve: serial componentwise oracle (numpy/scipy, FP64, "
                         f"1 thread, plain start{', tail estimate' if args.tail_estimate else ''}, the headline's "
                         f"stop rule), eps {args.eps}, {t_or:.2f} s",
               "time_to_1e-6_ms": round(t_or * 1e3, 1), "host_cores_available": len(os.sched_getaffinity(0)),
               "cpu_model": cpu_model()}
        log(f"cpu oracle {t_or:.2f}s")

    times = {name: round(ms, 4) for name, (ms, _, _) in res.items()}
    times["componentwise_cold"] = round(ms_cold, 4)
    times["componentwise_device_eager"] = round(mcw["kernel_ms"], 4)
    times["plain_plain_stop_device_eager"] = round(mpl["kernel_ms"], 4)
    times["componentwise_eager_with_launch_events"] = round(t_ecw / args.steps * 1e3, 4)
    times["plain_plain_stop_eager_with_launch_events"] = round(t_epl / args.steps * 1e3, 4)
    stop_rule = "the tail-estimate stop" if args.tail_estimate else "the 1-norm stop"
    out = {
        "metric": METRIC,
        "value": round(value, 4),
        "unit": "GEdge-iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_cw, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if args.precision == 0 else "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.config}: {'Barabasi-Albert' if 'ba_' in args.config else 'web-like'} "
                               f"graph n={g.n} m={g.m}, c={args.c}, "
                               f"1-norm certificate eps={args.eps}, W=1, componentwise solve with {stop_rule} "
                               f"and the FP64 residual certificate, plan resident",
                   "n": g.n, "m": g.m, "levels": info["n_levels"], "components": info["n_comp"],
                   "scc": info["n_scc"], "scc_vertices": info["v_scc"], "m_scc_internal": info["m_scc_internal"],
                   "m_between": info["m_between"], "m_cac_internal": info["m_cac_internal"],
                   "gang_vertices": info["v_gang"], "rows_per_wave": info["rows_per_wave"],
                   "small_cutoff": info["small_cutoff"], "team_edges": info["team_edges"],
                   "grid_wgs": info["grid_wgs"], "seg_waves": info["seg_waves"], "hipgraph": bool(args.graph),
                   "tail_estimate": bool(args.tail_estimate),
                   "autotuned": bool(bopts.get("autotune", 0))},
        "time_to_1e-6_ms": times,
        # like for like: both methods with the same stop rule
        "speedup_vs_plain": round(ms_pl / ms_cw, 3),
        "speedup_vs_plain_both_plain_stop": round(ms_pl_nt / ms_cw_nt, 3),
        "plain_gedge_iter_s": round(sp_nt["edge_iters"] / (ms_pl_nt * 1e-3) / 1e9, 4),
        "plain_equivalent_gedge_iter_s": round(sp_nt["edge_iters"] / (ms_cw * 1e-3) / 1e9, 4),
        "iterations": {name: {"terms_max": st["iters_max"], "terms_sum": st["iters_sum"],
                              "edge_iters": st["edge_iters"], "refine_rounds": st["refine_rounds"]}
                       for name, (_, st, _) in res.items()},
        "starting_guess": None if net is None else {
            "network": os.path.relpath(args.warm_net, ROOT),
            "kept": res["componentwise_guess"][1]["ws_accepted"],
            "fell_back": res["componentwise_guess"][1]["ws_rejected"],
            "not_in_headline": "with the tail-estimate stop the guess saves no series terms and costs its passes"},
        "rel_l1_vs_fp64_oracle": acc,
        "partition_ms": round(t_part * 1e3, 2),
        "build_ms": round(t_build * 1e3, 2),
        "kernel_times": kt,
        "roofline": roof,
        "roofline_spmv": roof_spmv,
        "cpu_baseline": cpu,
        "device": dev_name,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
