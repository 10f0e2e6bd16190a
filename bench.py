"""Benchmark: componentwise PageRank vs plain power series on one MI355X.

One step = one pr_solve of the componentwise method (Sec. 3.3: boundary
mass, one-vertex components, CAC sweeps, SCC power series, output) on the
web-like graph of 1M vertices / 10M edges, with the plan resident on the
device.  The plain whole-graph power series (Sec. 4.2, method 1) is timed the
same way as the comparator.  Both stop on the 1-norm certificate at 1e-6.

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

# algorithmic bytes: series terms FP32 (mixed) or FP64
B_EDGE_ITER = {0: 8, 1: 12}       # source index + term gather
B_VERT_ITER = {0: 28, 1: 36}      # row ptr, 1/outdeg, term write, R read+write
B_EDGE_ONCE = 12                  # between/CAC edge: source index + x gather
B_VERT_ONCE = 44                  # W, perm, two row ptrs, R out, x, 1/outdeg


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def alg_bytes(st, info, prec, plain):
    b = st["edge_iters"] * 0
    if plain:
        b = st["edge_iters"] * B_EDGE_ITER[prec] + st["vert_iters"] * B_VERT_ITER[prec]
        b += info["n"] * 28
        return b
    e_once = info["m_between"] + info["m_cac_internal"]
    e_it = st["edge_iters"] - e_once
    v_once = info["n"]
    v_it = st["vert_iters"] - (info["n"] - info["v_scc"])
    return e_it * B_EDGE_ITER[prec] + v_it * B_VERT_ITER[prec] + e_once * B_EDGE_ONCE + v_once * B_VERT_ONCE


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
    ap.add_argument("--graph", type=int, default=0, help="replay a captured hipGraph")
    ap.add_argument("--rows-per-wave", type=int, default=0)
    ap.add_argument("--small-cutoff", type=int, default=0)
    ap.add_argument("--team-edges", type=int, default=0)
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="also run a plain device copy of this size (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only; --gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1609_09068_amd as pr
    from graphgen import config_graph

    torch.cuda.set_device(0)
    dev_name = torch.cuda.get_device_name(0)
    log("device", dev_name)
    t0 = time.perf_counter()
    g = config_graph(args.config)
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
    common = dict(eps=args.eps, precision=args.precision, use_graph=args.graph)

    def run(method, Rout, steps):
        stats = []
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            rc, st = pr.pr_solve(lv, args.c, W, Rout, method=method, **common)
            stats.append(st)
        torch.cuda.synchronize()
        return (time.perf_counter() - t), stats

    for _ in range(args.warmup):
        run(0, R, 1)
        run(1, Rp, 1)
    log("warmup done")
    t_cw, st_cw = run(0, R, args.steps)
    log(f"componentwise: {t_cw / args.steps * 1e3:.3f} ms/step")
    t_pl, st_pl = run(1, Rp, args.steps)
    log(f"plain: {t_pl / args.steps * 1e3:.3f} ms/step")

    if args.calib_copy_mb:
        nb = args.calib_copy_mb * (1 << 20) // 4
        a = torch.ones(nb, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log(f"calibration copy: {args.calib_copy_mb} MiB read + {args.calib_copy_mb} MiB write")

    # accuracy against the FP64 oracle reference
    from oracle.pagerank import pagerank_power_series

    t0 = time.perf_counter()
    ref, kref, _ = pagerank_power_series(g.n, g.row_ptr, g.col, args.c, np.ones(g.n), eps=1e-12)
    log(f"oracle reference (eps 1e-12, {kref} iterations) {time.perf_counter() - t0:.1f}s")
    Rc = R.cpu().numpy()
    Rpl = Rp.cpu().numpy()
    err_cw = float(np.abs(Rc - ref).sum() / ref.sum())
    err_pl = float(np.abs(Rpl - ref).sum() / ref.sum())
    ref_part = None

    ms_cw = t_cw / args.steps * 1e3
    ms_pl = t_pl / args.steps * 1e3
    s = st_cw[-1]
    sp = st_pl[-1]
    kms_cw = float(np.mean([x["kernel_ms"] for x in st_cw]))
    kms_pl = float(np.mean([x["kernel_ms"] for x in st_pl]))
    value = s["edge_iters"] / (ms_cw * 1e-3) / 1e9
    bytes_cw = alg_bytes(s, info, args.precision, False)
    bytes_pl = alg_bytes(sp, info, args.precision, True)
    ach_cw = bytes_cw / (kms_cw * 1e-3) / 1e9
    ach_pl = bytes_pl / (kms_pl * 1e-3) / 1e9

    cpu = None
    if not args.no_cpu:
        from threadpoolctl import threadpool_limits

        from oracle.componentwise import componentwise_solve

        with threadpool_limits(limits=1):
            t0 = time.perf_counter()
            Ro, sto = componentwise_solve(g.n, g.row_ptr, g.col, args.c, np.ones(g.n), eps=args.eps,
                                          return_stats=True)
            t_or = time.perf_counter() - t0
        part_d = part.as_dict()
        scc = part_d["comp_type"] == 1
        e_int = np.zeros(part.n_comp)
        # internal edges per SCC from the oracle's own partition arrays
        src = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
        keep = (src != g.col) & (part_d["comp"][src] == part_d["comp"][g.col])
        np.add.at(e_int, part_d["comp"][src[keep]], 1)
        e_iter_or = float(np.sum(sto["iters"][scc] * e_int[scc])) + (info["m_between"] + info["m_cac_internal"])
        cpu = {"value": e_iter_or / t_or / 1e9, "unit": "GEdge-iter/s", "cores": 1, "kind": "oracle",
               "sample": f"full {args.config} graph, serial componentwise oracle (numpy/scipy FP64, "
                         f"1 thread), eps {args.eps}: {t_or:.2f} s",
               "time_to_1e-6_ms": t_or * 1e3, "host_cores_available": len(os.sched_getaffinity(0))}
        log(f"cpu oracle {t_or:.2f}s")

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
        "config": {"workload": f"{args.config}: web-like graph n={g.n} m={g.m}, c={args.c}, "
                               f"1-norm certificate eps={args.eps}, W=1, solve with plan resident",
                   "n": g.n, "m": g.m, "levels": info["n_levels"], "components": info["n_comp"],
                   "scc": info["n_scc"], "scc_vertices": info["v_scc"], "m_scc_internal": info["m_scc_internal"],
                   "m_between": info["m_between"], "m_cac_internal": info["m_cac_internal"],
                   "rows_per_wave": info["rows_per_wave"], "small_cutoff": info["small_cutoff"],
                   "team_edges": info["team_edges"], "grid_wgs": info["grid_wgs"], "hipgraph": bool(args.graph)},
        "time_to_1e-6_ms": {"componentwise": round(ms_cw, 4), "plain": round(ms_pl, 4),
                            "componentwise_kernel": round(kms_cw, 4), "plain_kernel": round(kms_pl, 4)},
        "speedup_vs_plain": round(ms_pl / ms_cw, 3),
        "plain_gedge_iter_s": round(sp["edge_iters"] / (ms_pl * 1e-3) / 1e9, 4),
        "plain_equivalent_gedge_iter_s": round(sp["edge_iters"] / (ms_cw * 1e-3) / 1e9, 4),
        "iterations": {"componentwise_max": s["iters_max"], "plain": sp["iters_max"],
                       "edge_iters_cw": s["edge_iters"], "edge_iters_plain": sp["edge_iters"]},
        "rel_l1_vs_fp64_oracle": {"componentwise": err_cw, "plain": err_pl,
                                  "cert_componentwise": s["cert_rel"], "cert_plain": sp["cert_rel"]},
        "partition_ms": round(t_part * 1e3, 2),
        "build_ms": round(t_build * 1e3, 2),
        "roofline": {"bound": "hbm", "achieved": round(ach_cw, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(ach_cw / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "k_solve (componentwise)", "alg_bytes_per_launch": int(bytes_cw),
                     "kernel_ms": round(kms_cw, 4),
                     "plain": {"achieved": round(ach_pl, 2), "frac": round(ach_pl / HBM_PEAK_GBS, 4),
                               "alg_bytes_per_launch": int(bytes_pl), "kernel_ms": round(kms_pl, 4)}},
        "cpu_baseline": cpu,
        "device": dev_name,
    }
    del ref_part
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
