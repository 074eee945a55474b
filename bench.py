"""Throughput of the restarted-PDHG hot path on one MI355X.

A step is one check window: 64 accepted PDHG iterations (both sparse products
with their fused dual/primal/averaging epilogues, the step-size tests, and the
termination/restart check that closes the window) on the 2e6-variable,
1e6-row, ~2e7-nonzero synthetic LP in FP64 (--workload pagerank: the LP of
the PageRank vector of a random 1e6-node graph, m = n + 1, ~8e6 nonzeros, one
dense row).  The timed region is one lp_solve
of K windows that starts after W warm-up windows; problem data and iterates
are resident in HBM before it starts (load and scaling are excluded, as in the
paper's timings).

Besides the JSON fields of the harness contract the line carries:
  roofline      the dominant kernel's algorithmic bytes per launch divided by
                its mean hipEvent duration, against the 8 TB/s HBM peak.  The
                events bracket every launch of the timed region's first window
                (64 launch pairs, plain launches); the other windows replay the
                captured graph, as an untimed solve does (--kernel-timing 1:
                events in every window).  `traffic` is the counter-measured HBM
                bytes per launch from profiles/ (null when the kernel changed
                since)
  spmv          the same figure for both SpMV kernels
  cpu_baseline  the FP64 CPU oracle on a bounded sample of the same instance
  time_to_tol   wall time of a cold solve to relative KKT error 1e-4 (--ttt-tol)
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

ITERS_PER_STEP = 64
HBM_PEAK_GBS = 8000.0
def kernel_names(precision):
    t = "double" if precision == "fp64" else "float"
    return {0: f"k_partial_K<{t}>+k_dual<{t}>", 1: f"k_partial_KT<{t}>+k_update<{t}>"}


def kernel_bytes(which, n, m, nnz, s=8):
    """Algorithmic bytes of one launch of the fused SpMV kernels (accepted
    step, no check in the window): streamed matrix values and indices, row
    pointers, the gathered vector counted once, and every vector the epilogue
    reads or writes."""
    if which == 0:   # K x' + dual update: reads y, Kx, q; writes y', Kx'
        return nnz * (s + 4) + 4 * (m + 1) + s * n + 5 * s * m
    # K'y' + averages + next primal: columns read x', c, l, u, xbar, K'ybar and
    # write K'y', xbar, K'ybar, x''; rows read y', Kx', ybar, Kxbar, write ybar, Kxbar
    return nnz * (s + 4) + 4 * (n + 1) + s * m + 10 * s * n + 6 * s * m


def kernel_source_sha():
    h = hashlib.sha256()
    for f in ("kernels.hip", "device.h", "internal.h"):
        with open(os.path.join(ROOT, "paper_2312_14832_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def counter_traffic(kernel, workload, layout=None):
    """HBM bytes per launch from the committed counter summary, if it was
    taken on the current kernel source and on the same layout (column
    slices, nonzeros and rows per row block of K and K')."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    e = d.get(workload, {}).get(kernel)
    if not e or e.get("source_sha") != kernel_source_sha():
        return None
    if layout is not None and e.get("layout") != layout:
        return None
    return e.get("traffic_bytes")


def profiled_layout(dirpath):
    """Layout of a profiled run, from the bench's own line in DIR/stats.log
    (the profile commands run with --autotune 0, so the row blocks are the
    default 2048 nonzeros and 1024 rows unless the line names them)."""
    import re
    text = open(os.path.join(dirpath, "stats.log")).read()
    m = re.search(r"layout K \(S, nnz/block, rows/block, split sums\) = \((\d+), (\d+), (\d+), (\d+)\), "
                  r"K' = \((\d+), (\d+), (\d+), (\d+)\)", text)
    if m:
        v = [int(g) for g in m.groups()]
        return {"K": v[:4], "KT": v[4:]}
    m = re.search(r"layout K \(S, nnz/block, rows/block\) = \((\d+), (\d+), (\d+)\), "
                  r"K' = \((\d+), (\d+), (\d+)\)", text)
    if m:
        v = [int(g) for g in m.groups()]
        return {"K": v[:3], "KT": v[3:]}
    m = re.search(r"column slices \(K, K'\) = \((\d+), (\d+)\)", text)
    if not m:
        return None
    return {"K": [int(m.group(1)), 2048, 1024], "KT": [int(m.group(2)), 2048, 1024]}


def _kernel_short(name):
    base = name.split("(")[0]
    if base.startswith("void "):
        base = base[5:]
    return base[len("pdlp::"):] if base.startswith("pdlp::") else base


def _counter_avgs(db, counter):
    import sqlite3
    con = sqlite3.connect(db)
    rows = con.execute("select kernel_name, count(*), avg(value) from counters_collection "
                       "where counter_name = ? group by kernel_name", (counter,)).fetchall()
    con.close()
    return {_kernel_short(k): (cnt, avg) for k, cnt, avg in rows}


def _durations(db):
    import sqlite3
    con = sqlite3.connect(db)
    rows = con.execute("select name, count(*), avg(duration), sum(duration) from kernels group by name").fetchall()
    con.close()
    return {_kernel_short(k): (cnt, avg, tot) for k, cnt, avg, tot in rows}


def traffic_from(dirpath, precision, workload, copy_bytes):
    """Per-launch HBM traffic of the two fused SpMV kernel pairs from rocprofv3
    FETCH_SIZE / WRITE_SIZE runs (KiB per dispatch), each scaled by what the
    same counter reads for a device-to-device copy of `copy_bytes`; written to
    profiles/traffic.json under the current kernel source hash.  Prints a
    markdown summary of durations and counters."""
    db = lambda sub: os.path.join(dirpath, sub, "run_results.db")
    fetch, write = _counter_avgs(db("fetch"), "FETCH_SIZE"), _counter_avgs(db("write"), "WRITE_SIZE")
    cf, cw = _counter_avgs(db("copy_fetch"), "FETCH_SIZE"), _counter_avgs(db("copy_write"), "WRITE_SIZE")
    copy = "__amd_rocclr_copyBuffer"
    ff = copy_bytes / (cf[copy][1] * 1024.0)
    wf = copy_bytes / (cw[copy][1] * 1024.0)
    stats = _durations(db("stats")) if os.path.exists(db("stats")) else {}
    path = os.path.join(ROOT, "profiles", "traffic.json")
    d = json.load(open(path)) if os.path.exists(path) else {}
    d[workload] = {}
    sha = kernel_source_sha()
    lines = [f"copy calibration ({copy_bytes} B per copy): FETCH_SIZE x{ff:.4f}, WRITE_SIZE x{wf:.4f}", "",
             "| kernel | launches | avg us | FETCH KiB | WRITE KiB | scaled MB/launch |", "|---|---|---|---|---|---|"]
    def find(table, label):
        # 'k_dual<double>' names every instantiation 'k_dual<double, S>'
        stem = label[:-1]
        hits = [k for k in table if k == label or k.startswith(stem + ",")]
        assert len(hits) == 1, (label, hits)
        return table[hits[0]], hits[0]

    layout = profiled_layout(dirpath) if os.path.exists(os.path.join(dirpath, "stats.log")) else None
    for pair in kernel_names(precision).values():
        e = {"source_sha": sha, "fetch_factor": ff, "write_factor": wf, "layout": layout, "parts": {}}
        tot = 0.0
        for k in pair.split("+"):
            (_, fk), full = find(fetch, k)
            (_, wk), _ = find(write, k)
            b = fk * 1024.0 * ff + wk * 1024.0 * wf
            tot += b
            e["parts"][full] = {"fetch_kib": fk, "write_kib": wk, "traffic_bytes": b}
            cnt, avg, _ = stats.get(full, (0, float("nan"), 0))
            lines.append(f"| {full} | {cnt} | {avg / 1e3:.1f} | {fk:.0f} | {wk:.0f} | {b / 1e6:.0f} |")
        e["traffic_bytes"] = tot
        d[workload][pair] = e
    with open(path, "w") as f:
        json.dump(d, f, indent=1)
        f.write("\n")
    if stats:
        lines += ["", "| kernel (all) | launches | avg us | total ms |", "|---|---|---|---|"]
        for k, (cnt, avg, tot) in sorted(stats.items(), key=lambda kv: -kv[1][2])[:12]:
            lines.append(f"| {k} | {cnt} | {avg / 1e3:.1f} | {tot / 1e6:.2f} |")
    print("\n".join(lines))


def compare_with_fp64(lp, data, prob, ttt, stream, args):
    """Error of the mixed-precision result against FP64: its KKT quantities
    evaluated in FP64 on the GPU (an FP64 handle started at the mixed point,
    zero iterations), and the objective against an FP64 solve to the same
    tolerance."""
    import torch
    x, y, _, _ = prob.result()
    p64 = lp.Problem(data, precision="fp64", stream=stream)
    p64.set_start(x, y)
    eps = args.ttt_tol
    ev = p64.solve(eps, 0)
    t0 = time.perf_counter()
    p64.set_start(None, None)
    ref = p64.solve(eps, 10**7, args.ttt_limit)
    torch.cuda.synchronize()
    t64 = time.perf_counter() - t0
    p64.close()
    out = {"fp64_eval_of_mixed_point": {"rel_primal": ev["rel_primal"], "rel_dual": ev["rel_dual"],
                                        "rel_gap": ev["rel_gap"], "rel_kkt": ev["rel_kkt"], "pobj": ev["pobj"]},
           "fp64_solve": {"status": ref["status"], "iterations": ref["iterations"], "seconds": t64,
                          "pobj": ref["pobj"], "rel_kkt": ref["rel_kkt"]},
           "objective_rel_diff": abs(ttt["pobj"] - ref["pobj"]) / max(1.0, abs(ref["pobj"]))}
    print(f"[bench] mixed point in FP64: rel KKT {ev['rel_kkt']:.3e}; objective vs FP64 solve "
          f"{out['objective_rel_diff']:.2e} (FP64 solve {t64:.2f}s, {ref['iterations']} it)",
          file=sys.stderr, flush=True)
    return out


def cpu_baseline(data, max_windows=3, budget_s=13.0):
    """The single-threaded FP64 oracle on the same instance: one 64-step
    window is timed to size the sample, then (if more than one window fits
    in budget_s, up to max_windows) one solve of that many windows from the
    start is the sample.  Every oracle solve starts from the start point."""
    from oracle.oracle import Oracle
    o = Oracle(data)
    t = time.perf_counter()
    o.solve(1e-30, ITERS_PER_STEP)
    dt = time.perf_counter() - t
    windows = max(1, min(max_windows, int(budget_s // max(dt, 1e-9))))
    if windows > 1:
        t = time.perf_counter()
        o.solve(1e-30, windows * ITERS_PER_STEP)
        dt = time.perf_counter() - t
    iters = windows * ITERS_PER_STEP
    return {"value": iters / dt, "unit": "PDHG iters/sec", "cores": 1, "kind": "oracle",
            "sample": f"{iters} accepted iterations ({windows} check windows incl. start-up products) "
                      f"of the single-threaded FP64 oracle on the same instance, load and scaling excluded",
            "seconds": dt}


def host_cpu_model():
    """The host CPU's model name (from /proc/cpuinfo; "unknown" elsewhere)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def workload_name(args):
    """Key of a single-LP workload in the bench line and in traffic.json."""
    base = f"pagerank_lp_n{args.n}" if args.workload == "pagerank" else f"large_powerlaw_lp_n{args.n}"
    return base + ("" if args.precision == "fp64" else "_mixed")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=None,
                    help="variables (large: 2,000,000; pagerank: 1,000,000 graph nodes)")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--no-ttt", action="store_true", help="skip the time-to-tolerance solve")
    ap.add_argument("--no-other-configs", action="store_true",
                    help="default workload: skip the short runs of the tiny, mixed-precision and batched "
                         "configurations that the line carries under other_configs")
    ap.add_argument("--ttt-tol", type=float, default=1e-4, help="relative KKT tolerance of that solve")
    ap.add_argument("--ttt-limit", type=float, default=90.0)
    ap.add_argument("--ws-train", type=int, default=2048, help="warmstart: training instances")
    ap.add_argument("--ws-eval", type=int, default=1000, help="warmstart: held-out instances")
    ap.add_argument("--ws-label-precision", choices=["fp64", "mixed"], default="fp64",
                    help="warmstart: precision of the label solves (mixed: FP32 products, every label's 1e-5 "
                         "confirmed by the FP64 re-check)")
    ap.add_argument("--ws-epochs", type=int, default=120)
    ap.add_argument("--ws-time-sample", type=int, default=64,
                    help="warmstart: held-out members also timed one by one on single handles")
    ap.add_argument("--workload", choices=["large", "pagerank", "tiny", "batch", "warmstart", "gemm", "shared", "gather"],
                    default="large",
                    help="large: one 2e6x1e6 LP (default); pagerank: the LP of a random graph's PageRank "
                         "vector; batch: 512 uneven LPs solved together; shared: members of the warm-start "
                         "family solved over one shared matrix")
    ap.add_argument("--shared-count", type=int, default=64, help="shared: instances per handle")
    ap.add_argument("--batch-count", type=int, default=512)
    ap.add_argument("--batch-kind", choices=["uneven", "tiny"], default="uneven",
                    help="batch: 512 uneven LPs (n 2e3..2e5, to 1e-4) or 512 tiny LPs (n=1000, to 1e-6)")
    ap.add_argument("--batch-fixed-iters", type=int, default=0,
                    help="batch: only a fixed number of iterations with every instance active (profiling)")
    ap.add_argument("--seq-sample", type=int, default=128,
                    help="batch workload: instances solved one by one for the sequential comparison")
    ap.add_argument("--kernel-timing", type=int, default=2, choices=[0, 1, 2],
                    help="2: HIP events around the two fused products in the first window of the timed "
                         "region, the other windows replaying the captured graph (roofline; default); "
                         "1: events in every window (plain launches); 0: no events")
    ap.add_argument("--autotune", type=int, default=1, choices=[0, 1],
                    help="1: time neighbouring layouts at load and keep the fastest; 0: the default layout")
    ap.add_argument("--split-sums", type=int, default=-1, choices=[-1, 0, 1],
                    help="row sums of short-row blocks: 1 split by entries, 0 one row per thread, -1 the "
                         "library's default (split; with --autotune 1 the other form is timed per product)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run 5 plain device-to-device copies of this many MiB (counter calibration)")
    ap.add_argument("--traffic-from", default=None,
                    help="no GPU: read rocprofv3 databases under DIR/{stats,fetch,write,copy_fetch,copy_write} "
                         "and write profiles/traffic.json for the chosen single-LP workload")
    ap.add_argument("--copy-mib", type=int, default=1024, help="size of the calibration copy for --traffic-from")
    args = ap.parse_args()
    if args.n is None:
        args.n = 1_000_000 if args.workload == "pagerank" else 2_000_000
    if args.traffic_from:
        return traffic_from(args.traffic_from, args.precision, workload_name(args), args.copy_mib << 20)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              f"(sharding over several GPUs is not implemented)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2312_14832_amd import gen, lp

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_probe_mib:
        nbytes = args.copy_probe_mib << 20
        a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": nbytes, "copies": 5}))
        return
    if args.workload == "batch":
        return bench_batch(args)
    if args.workload == "tiny":
        return bench_tiny(args)
    if args.workload == "gemm":
        return bench_gemm(args)
    if args.workload == "warmstart":
        return bench_warmstart(args)
    if args.workload == "shared":
        return bench_shared(args)
    if args.workload == "gather":
        return bench_gather(args)
    n = args.n
    t0 = time.perf_counter()
    if args.workload == "pagerank":
        data = gen.pagerank_lp(seed=args.seed, n=n)
        recipe = ("random graph, 1 + Poisson(5) links per node (repeats collapsed), damping 0.85; "
                  "row 0: sum(x) = 1, rows 1..n: x - 0.85 A x >= 0.15/n, x >= 0, c = 0")
    else:
        data = gen.large_lp(seed=args.seed, n=n, m1=n // 4, m2=n // 4)
        recipe = ("power-law column counts 1..200 (mean 10), N(0,1)*10^U(-3,3) per row, "
                  "certificate-feasible")
    workload = workload_name(args)
    m1, m2 = data.m1, data.m - data.m1
    gen_s = time.perf_counter() - t0
    print(f"[bench] generated n={n} m={m1 + m2} nnz={data.nnz} in {gen_s:.1f}s", file=sys.stderr, flush=True)

    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    prob = lp.Problem(data, precision=args.precision, stream=stream, kernel_timing=args.kernel_timing,
                      autotune=args.autotune, split_sums=args.split_sums)
    torch.cuda.synchronize()
    load_s = time.perf_counter() - t0
    lk, lt = (prob.layout_blocks(w) + (prob.layout_split(w),) for w in (0, 1))
    print(f"[bench] loaded in {load_s:.1f}s ({prob.device_bytes() / 2**30:.2f} GiB on device), "
          f"column slices (K, K') = {prob.layout()}; layout K (S, nnz/block, rows/block, split sums) = {lk}, "
          f"K' = {lt}", file=sys.stderr, flush=True)

    # warm-up windows (also compiles nothing: kernels are prebuilt)
    prob.solve(1e-30, ITERS_PER_STEP * max(args.warmup, 0))
    torch.cuda.synchronize()

    K = args.steps
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = prob.solve(1e-30, ITERS_PER_STEP * K)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    iters = info["iterations"]
    assert iters == ITERS_PER_STEP * K, info
    s = 8 if args.precision == "fp64" else 4
    spmv = {}
    for w in (0, 1):
        cnt, ms = prob.kernel_time(w)
        avg_us = 1e3 * ms / max(cnt, 1)
        b = kernel_bytes(w, n, m1 + m2, data.nnz, s)
        spmv[kernel_names(args.precision)[w]] = {"launches": cnt, "avg_us": avg_us, "alg_bytes": b,
                                 "GB_s": b / (avg_us * 1e-6) / 1e9 if avg_us > 0 else None,
                                 "gathers": data.nnz,
                                 "G_gathers_s": data.nnz / (avg_us * 1e-6) / 1e9 if avg_us > 0 else None}
    dom = max(spmv, key=lambda k: spmv[k]["avg_us"] * spmv[k]["launches"])
    d = spmv[dom]
    roofline = {"kernel": dom, "bound": "hbm", "achieved": d["GB_s"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": d["GB_s"] / HBM_PEAK_GBS if d["GB_s"] else None,
                "traffic": counter_traffic(dom, workload, {"K": list(lk), "KT": list(lt)}),
                "alg_bytes_per_launch": d["alg_bytes"],
                "timed_launches": d["launches"]}
    # the gather ceiling at the dominant product's layout (lp_gather_probe: i.i.d.
    # columns over the same slices, dealt to the XCDs the same way)
    gather_roofline = None
    try:
        import numpy as np
        wdom = list(spmv).index(dom)
        S_dom = prob.layout()[wdom]
        vec_len = n if wdom == 0 else m1 + m2
        slice_len = (vec_len + S_dom - 1) // S_dom
        per = data.nnz // S_dom
        grng = np.random.Generator(np.random.PCG64(11))
        gidx = torch.from_numpy(grng.integers(0, slice_len, size=per * S_dom).astype(np.int32)).cuda()
        gx = torch.ones(S_dom * slice_len, dtype=torch.float64 if s == 8 else torch.float32, device="cuda")
        gms = lp.gather_probe(gidx, gx, S_dom, slice_len, reps=20)
        ceiling = per * S_dom / (gms * 1e-3) / 1e9
        gather_roofline = {"kernel": dom, "bound": "gathers", "achieved": d["G_gathers_s"], "peak": ceiling,
                           "unit": "G gathers/s", "frac": d["G_gathers_s"] / ceiling,
                           "peak_source": f"lp_gather_probe: {per * S_dom} i.i.d. gathers over {S_dom} slices of "
                                          f"{slice_len} entries, measured in this run"}
        del gidx, gx
    except Exception as exc:   # the probe is context; the bench line stands without it
        print(f"[bench] gather probe skipped: {exc}", file=sys.stderr, flush=True)
    print(f"[bench] {K} windows in {dt:.3f}s -> {iters / dt:.0f} it/s; "
          + "; ".join(f"{k} {v['avg_us']:.1f}us {v['GB_s'] or 0:.0f}GB/s" for k, v in spmv.items()),
          file=sys.stderr, flush=True)

    prob_layout = prob.layout()
    blocks = {name: dict(zip(("slices", "nnz_per_block", "rows_per_block", "split_sums"),
                             prob.layout_blocks(w) + (prob.layout_split(w),)))
              for w, name in ((0, "K"), (1, "KT"))}
    ttt = None
    if not args.no_ttt:
        t0 = time.perf_counter()
        tinfo = prob.solve(args.ttt_tol, 10**7, args.ttt_limit)
        torch.cuda.synchronize()
        tt = time.perf_counter() - t0
        ttt = {"tol": args.ttt_tol, "seconds": tt, "status": tinfo["status"], "iterations": tinfo["iterations"],
               "attempts": tinfo["attempts"], "restarts": tinfo["restarts"], "rel_kkt": tinfo["rel_kkt"],
               "pobj": tinfo["pobj"], "time_limit_s": args.ttt_limit}
        print(f"[bench] time to {args.ttt_tol:g}: {tt:.2f}s {tinfo['status']} after {tinfo['iterations']} iterations",
              file=sys.stderr, flush=True)
    mixed_vs_fp64 = None
    if not args.no_ttt and args.precision == "mixed":
        mixed_vs_fp64 = compare_with_fp64(lp, data, prob, ttt, stream, args)
    prob.close()

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(data)   # about 13 s of one host core on the default workload
        cpu["threads_note"] = f"host has {os.cpu_count()} logical CPUs; the oracle is single-threaded"
        cpu["cpu_model"] = host_cpu_model()
        print(f"[bench] cpu oracle {cpu['value']:.2f} it/s", file=sys.stderr, flush=True)

    out = {
        "metric": "PDHG iters/sec",
        "value": iters / dt,
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * dt / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64acc",
        "data": "synthetic",
        "config": {"workload": workload, "n": n, "m1": m1, "m2": m2, "nnz": data.nnz, "seed": args.seed,
                   "precision": args.precision, "iters_per_step": ITERS_PER_STEP,
                   "column_slices": list(prob_layout), "row_blocks": blocks,
                   "generator": recipe},
        "roofline": roofline,
        "gather_roofline": gather_roofline,
        "spmv": spmv,
        "time_to_tol": ttt,
        "mixed_vs_fp64": mixed_vs_fp64,
        "cpu_baseline": cpu,
        "load_s": load_s,
        "gen_s": gen_s,
    }
    if (args.workload == "large" and args.n == 2_000_000 and args.precision == "fp64" and not args.no_ttt
            and not args.no_other_configs):
        out["other_configs"] = other_configs(args)
    print(json.dumps(out))


def other_configs(args):
    """Short runs of the other configurations, so that one default bench run
    measures them all: the tiny LPs (one-workgroup loop and launches, time to
    1e-6, the oracle's time beside them), the 4e6-column LP in mixed precision
    (iteration rate, time to 1e-4, the returned point evaluated in FP64), the
    batch of 512 uneven LPs (time to 1e-4, against a sample of them solved one
    by one), and a batch of 512 tiny LPs (one workgroup per LP, the batched
    launches, 32 of them one by one).  Each result is in the unit of its own
    configuration."""
    import torch
    res = {}
    print("[bench] other configurations: tiny", file=sys.stderr, flush=True)
    t = run_tiny(args, steps=20, warmup=2, with_cpu=True)
    res[t["config"]["workload"]] = {k: t[k] for k in ("metric", "value", "unit", "dtype", "config", "time_to_tol",
                                                      "forms", "cpu_baseline")}
    torch.cuda.empty_cache()
    print("[bench] other configurations: mixed precision, n = 4e6", file=sys.stderr, flush=True)
    res["large_powerlaw_lp_n4000000_mixed"] = run_mixed_short(args)
    torch.cuda.empty_cache()
    print("[bench] other configurations: batch of 512", file=sys.stderr, flush=True)
    b = run_batch(args, precision="mixed", seq_sample=32)
    res[b["config"]["workload"] + "_mixed"] = {k: b[k] for k in ("metric", "value", "unit", "dtype", "config",
                                                                 "batch_seconds", "solved", "iterations_median",
                                                                 "iterations_max", "sequential")}
    torch.cuda.empty_cache()
    print("[bench] other configurations: batch of 512 tiny LPs", file=sys.stderr, flush=True)
    saved = (args.seq_sample, args.precision)
    args.seq_sample, args.precision = 32, "fp64"
    t = run_batch_tiny(args)
    args.seq_sample, args.precision = saved
    res[t["config"]["workload"]] = {k: t[k] for k in ("metric", "value", "unit", "dtype", "config", "forms",
                                                      "sequential")}
    torch.cuda.empty_cache()
    return res


def run_mixed_short(args):
    """The 4e6 x 2e6 power-law LP (seed 2) in mixed precision: 10 timed
    windows (after one warm-up), a cold solve to rel KKT 1e-4, and the
    returned point's criteria evaluated in FP64 (an FP64 handle started at it,
    zero iterations)."""
    import torch
    from paper_2312_14832_amd import gen, lp
    n = 4_000_000
    data = gen.large_lp(seed=2, n=n, m1=n // 4, m2=n // 4)
    st = torch.cuda.current_stream()
    prob = lp.Problem(data, precision="mixed", stream=st, kernel_timing=2)
    prob.solve(1e-30, ITERS_PER_STEP)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = prob.solve(1e-30, ITERS_PER_STEP * 10)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    pairs = {}
    for w in (0, 1):
        cnt, ms = prob.kernel_time(w)
        avg_us = 1e3 * ms / max(cnt, 1)
        b = kernel_bytes(w, n, data.m, data.nnz, 4)
        pairs[kernel_names("mixed")[w]] = {"avg_us": avg_us, "alg_bytes": b,
                                           "hbm_frac": b / (avg_us * 1e-6) / 1e9 / HBM_PEAK_GBS}
    t0 = time.perf_counter()
    tinfo = prob.solve(1e-4, 10**7, args.ttt_limit)
    torch.cuda.synchronize()
    tt = time.perf_counter() - t0
    x, y, _, _ = prob.result()
    prob.close()
    p64 = lp.Problem(data, precision="fp64", stream=st)
    p64.set_start(x, y)
    ev = p64.solve(1e-4, 0)
    p64.close()
    print(f"[bench] mixed 4e6: {info['iterations'] / dt:.0f} it/s; time to 1e-4 {tt:.2f}s {tinfo['status']} "
          f"({tinfo['iterations']} it); FP64 rel KKT of the point {ev['rel_kkt']:.3e}", file=sys.stderr, flush=True)
    return {"metric": "PDHG iters/sec", "value": info["iterations"] / dt, "unit": "iters/s",
            "dtype": "f32+f64acc",
            "config": {"workload": "large_powerlaw_lp_n4000000_mixed", "n": n, "m1": data.m1,
                       "m2": data.m - data.m1, "nnz": data.nnz, "seed": 2, "timed_windows": 10},
            "spmv": pairs,
            "time_to_tol": {"tol": 1e-4, "seconds": tt, "status": tinfo["status"],
                            "iterations": tinfo["iterations"]},
            "fp64_eval_of_point": {"rel_primal": ev["rel_primal"], "rel_dual": ev["rel_dual"],
                                   "rel_gap": ev["rel_gap"], "rel_kkt": ev["rel_kkt"]}}


def bench_tiny(args):
    """The tiny LP (n=1000, m1=200, m2=300, 5 nonzeros per column; seeds
    0..9).  Its data (about 0.2 MB) sits in L2, so the rate is set by launch
    and synchronisation latency, not by memory.  Both loop forms are timed:
    the one-workgroup loop (the default for LPs this small: one launch per
    window, workgroup barriers between the steps) and the seven launches per
    slot of captured graph windows.  Reported: the iteration rate, the time
    to rel KKT 1e-6 per instance (fresh handle, load excluded), and the
    oracle's time to 1e-6 on one host core."""
    print(json.dumps(run_tiny(args, args.steps, args.warmup, not args.no_cpu)))


def run_tiny(args, steps, warmup, with_cpu):
    """The tiny-LP measurements of bench_tiny, as a dict."""
    import numpy as np
    import torch
    from paper_2312_14832_amd import gen, lp

    lps = [gen.tiny_lp(s) for s in range(10)]
    st = torch.cuda.current_stream()
    forms = {}
    for name, pers in (("one_workgroup", 1), ("launches", 0)):
        p = lp.Problem(lps[0], stream=st, persistent=pers)
        p.solve(1e-30, ITERS_PER_STEP * max(warmup, 1))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = p.solve(1e-30, ITERS_PER_STEP * steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        p.close()
        ttt = []
        for s, data in enumerate(lps):
            q = lp.Problem(data, stream=st, persistent=pers)
            t0 = time.perf_counter()
            inf = q.solve(1e-6, 10**6)
            torch.cuda.synchronize()
            ttt.append({"seed": s, "seconds": time.perf_counter() - t0, "iterations": inf["iterations"],
                        "status": inf["status"]})
            q.close()
        med = float(np.median([t["seconds"] for t in ttt]))
        forms[name] = {"iters_per_s": info["iterations"] / dt, "ms_per_step": 1e3 * dt / steps,
                       "time_to_1e6_median_s": med, "runs": ttt}
        print(f"[bench] tiny, {name}: {info['iterations'] / dt:.0f} it/s, median time to 1e-6 {med * 1e3:.1f} ms",
              file=sys.stderr, flush=True)
    ora = []
    if with_cpu:
        from oracle.oracle import Oracle
        for s, data in enumerate(lps):
            o = Oracle(data)
            t0 = time.perf_counter()
            _, _, _, oi = o.solve(1e-6, 10**6)
            ora.append({"seed": s, "seconds": time.perf_counter() - t0, "iterations": oi["iterations"]})
        print(f"[bench] tiny, CPU oracle: median time to 1e-6 "
              f"{1e3 * float(np.median([o['seconds'] for o in ora])):.1f} ms", file=sys.stderr, flush=True)
    head = forms["one_workgroup"]
    out = {
        "metric": "PDHG iters/sec", "value": head["iters_per_s"], "unit": "iters/s", "n_gpus": 1,
        "steps": steps, "warmup": warmup, "ms_per_step": head["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "tiny_lp_n1000", "n": 1000, "m1": 200, "m2": 300, "nnz": lps[0].nnz,
                   "seeds": list(range(10)), "iters_per_step": ITERS_PER_STEP, "loop": "one workgroup"},
        "roofline": {"bound": "latency", "achieved": None, "peak": None, "unit": None, "frac": None,
                     "traffic": None,
                     "note": "0.2 MB of data per iteration, resident in L2: launch and barrier latency bound"},
        "time_to_tol": {"tol": 1e-6, "median_s": head["time_to_1e6_median_s"], "runs": head["runs"]},
        "forms": {k: {kk: vv for kk, vv in v.items() if kk != "runs"} for k, v in forms.items()},
        "cpu_baseline": ({"kind": "oracle", "cores": 1, "unit": "s to 1e-6",
                          "median_s": float(np.median([o["seconds"] for o in ora])), "runs": ora}
                         if ora else None),
    }
    return out


def bench_gemm(args):
    """The network's GEMM kernels (lpw_gemm) at large square sizes and at the
    network's own shapes, timed with HIP events on the current stream:
    TFLOP/s against the MFMA BF16 (2.5 PFLOP/s) and FP32 vector (157.3
    TFLOP/s) dense peaks, and the relative error against an FP32 product of
    the same rounded operands."""
    import torch
    from paper_2312_14832_amd import warmstart as ws
    peak = {"bf16": 2500.0, "fp32": 157.3}
    cases = [(4096, 4096, 4096, False, False, 20), (4096, 4096, 4096, False, True, 20),
             (4096, 4096, 4096, True, False, 20), (4096, 4096, 4096, True, True, 20),
             (8192, 8192, 8192, False, False, 5),
             (256, 1024, 1024, False, False, 20), (1024, 1024, 256, True, False, 20),
             (256, 300000, 64, False, False, 20)]
    gen_ = torch.Generator(device="cuda").manual_seed(0)
    rows = []
    for prec in ("bf16", "fp32"):
        dt = torch.bfloat16 if prec == "bf16" else torch.float32
        for M, N, K, ta, tb, reps in cases:
            A = torch.randn((K, M) if ta else (M, K), device="cuda", generator=gen_).to(dt).contiguous()
            B = torch.randn((N, K) if tb else (K, N), device="cuda", generator=gen_).to(dt).contiguous()
            for _ in range(3):
                C = ws.gemm(A, B, ta, tb, prec)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                C = ws.gemm(A, B, ta, tb, prec)
            e1.record()
            torch.cuda.synchronize()
            us = 1e3 * e0.elapsed_time(e1) / reps
            tf = 2.0 * M * N * K / (us * 1e-6) / 1e12
            ref = (A.float().t() if ta else A.float()) @ (B.float().t() if tb else B.float())
            err = float((C - ref).norm() / ref.norm())
            rows.append({"precision": prec, "M": M, "N": N, "K": K, "trans_a": ta, "trans_b": tb, "us": us,
                         "TFLOP_s": tf, "frac_of_peak": tf / peak[prec], "relerr": err})
            print(f"[bench] gemm {prec} {M}x{N}x{K} ta={ta}: {us:.1f} us {tf:.1f} TFLOP/s relerr {err:.1e}",
                  file=sys.stderr, flush=True)
    big = rows[0]
    out = {"metric": "GEMM TFLOP/s (network kernels)", "value": big["TFLOP_s"], "unit": "TFLOP/s", "n_gpus": 1,
           "steps": 20, "warmup": 3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "bf16 x bf16 -> f32", "data": "synthetic",
           "config": {"workload": "gemm_4096_bf16"},
           "roofline": {"bound": "mfma", "achieved": big["TFLOP_s"], "peak": peak["bf16"], "unit": "TFLOP/s",
                        "frac": big["frac_of_peak"], "traffic": None},
           "cases": rows}
    print(json.dumps(out))


def bench_batch(args):
    """Time to rel KKT 1e-4 of a batch of uneven LPs solved together, against
    solving the same instances one after another on the same GPU.

    Workload: `args.batch_count` members of the batched generator (seeds
    1000..), n log-uniform in [2e3, 2e5], m = n/2 split 2:3, 3..8 nonzeros per
    column; FP32 iterates with FP64 reductions (or FP64 with --precision
    fp64).  The sequential leg solves every (count/seq_sample)-th instance
    with the single-LP path (load excluded) and scales the sum up.
    """
    if args.batch_kind == "tiny":
        print(json.dumps(run_batch_tiny(args)))
        return
    if args.batch_fixed_iters <= 0:
        print(json.dumps(run_batch(args, args.precision, args.seq_sample)))
        return
    import torch
    lps, bt, shapes, alg, nnz, gen_s, load_s = _batch_setup(args, args.precision)
    # every instance runs to the same number of accepted steps: the profiling
    # workload.  Every instance is active in the first N slots; instances
    # with rejected attempts need more slots, in which fewer are active.
    t0 = time.perf_counter()
    bt.solve(1e-30, args.batch_fixed_iters)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    slots = max(bt.info(i)["attempts"] for i in range(len(lps)))
    print(json.dumps({"metric": "batch attempt slots per second (every instance to a fixed number of steps)",
                      "value": slots / dt, "unit": "slots/s", "n_gpus": 1,
                      "steps": args.batch_fixed_iters, "warmup": args.warmup,
                      "slots": slots, "full_slots": args.batch_fixed_iters,
                      "ms_per_step": 1e3 * dt / args.batch_fixed_iters, "higher_is_better": True,
                      "scaling": "weak", "vs_baseline": None,
                      "dtype": "f64" if args.precision == "fp64" else "f32+f64acc", "data": "synthetic",
                      "config": {"workload": f"batch_{len(lps)}_uneven_lps", "count": len(lps), "sum_nnz": nnz,
                                 "padded_n": sum((p.n + 255) // 256 * 256 for p in lps),
                                 "padded_m": sum((p.m + 255) // 256 * 256 for p in lps),
                                 "precision": args.precision},
                      "alg_bytes_per_launch": alg}))


def run_batch_tiny(args):
    """A batch of tiny LPs (the tiny generator, n=1000, m1=200, m2=300, 5
    nonzeros per column; seeds 2000..) solved to rel KKT 1e-6: one workgroup
    per instance (the default for such a batch), the batched launches
    (persistent = 0), and a sample solved one by one on single-LP handles
    (each on its own one-workgroup loop)."""
    import numpy as np
    import torch
    from paper_2312_14832_amd import gen, lp

    tol = 1e-6
    lps = [gen.tiny_lp(2000 + i) for i in range(args.batch_count)]
    st = torch.cuda.current_stream()
    forms = {}
    for name, pers in (("one_workgroup_per_lp", -1), ("launches", 0)):
        bt = lp.Batch(lps, precision=args.precision, stream=st, persistent=pers)
        bt.solve(1e-30, 64)   # warm-up (graph capture, caches)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        bt.solve(tol, 10**6, args.ttt_limit)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        infos = [bt.info(i) for i in range(len(lps))]
        its = np.array([d["iterations"] for d in infos])
        forms[name] = {"loop_form": bt.loop_form(), "seconds": dt,
                       "solved": sum(1 for d in infos if d["status"] == "OPTIMAL"),
                       "iterations_median": float(np.median(its)), "iterations_max": int(its.max())}
        print(f"[bench] tiny batch, {name}: {forms[name]['solved']}/{len(lps)} optimal in {dt:.3f}s "
              f"(iterations median {np.median(its):.0f}, max {its.max()})", file=sys.stderr, flush=True)
        bt.close()
    stride = max(1, len(lps) // max(args.seq_sample, 1))
    times = []
    for i in range(0, len(lps), stride):
        p = lp.Problem(lps[i], precision=args.precision, stream=st)
        p.solve(1e-30, 64)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        p.solve(tol, 10**6, args.ttt_limit)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t1)
        p.close()
    times = np.array(times)
    seq_est = float(times.sum()) * len(lps) / len(times)
    seq_err = len(lps) * float(np.std(times, ddof=1)) / np.sqrt(len(times)) if len(times) > 1 else None
    head = forms["one_workgroup_per_lp"]
    print(f"[bench] tiny batch, one by one: {len(times)} in {times.sum():.2f}s -> {seq_est:.1f}s for all "
          f"(speedup {seq_est / head['seconds']:.0f}x)", file=sys.stderr, flush=True)
    return {"metric": "batch time-to-1e-6 KKT", "value": len(lps) / head["seconds"], "unit": "LPs/s", "n_gpus": 1,
            "steps": 1, "warmup": 1, "ms_per_step": 1e3 * head["seconds"], "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None,
            "dtype": "f64" if args.precision == "fp64" else "f32+f64acc", "data": "synthetic",
            "config": {"workload": f"batch_{len(lps)}_tiny_lps", "count": len(lps), "n": 1000, "m1": 200, "m2": 300,
                       "seeds": [2000, 2000 + len(lps) - 1], "precision": args.precision, "tol": tol},
            "forms": forms,
            "sequential": {"sample": len(times), "stride": stride, "seconds_sample": float(times.sum()),
                           "seconds_extrapolated": seq_est, "seconds_extrapolated_stderr": seq_err,
                           "speedup": seq_est / head["seconds"]}}


def _batch_setup(args, precision):
    """Generate and load the batch, time nothing: (lps, handle, row-block
    shapes, algorithmic bytes per launch, sum nnz, generation and load
    seconds).  One warm-up solve of the handle is included."""
    import torch
    from paper_2312_14832_amd import gen, lp

    t0 = time.perf_counter()
    lps = [gen.batch_member(1000 + i) for i in range(args.batch_count)]
    gen_s = time.perf_counter() - t0
    nnz = sum(p.nnz for p in lps)
    print(f"[bench] generated {len(lps)} LPs, sum n={sum(p.n for p in lps)}, sum nnz={nnz} in {gen_s:.1f}s",
          file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    bt = lp.Batch(lps, precision=precision, stream=torch.cuda.current_stream(), autotune=args.autotune,
                  split_sums=args.split_sums)
    load_s = time.perf_counter() - t0
    shapes = {"K": bt.layout_blocks(0), "KT": bt.layout_blocks(1)}
    print(f"[bench] batch loaded in {load_s:.1f}s ({bt.device_bytes() / 2**30:.2f} GiB), row blocks "
          f"(nonzeros, rows) {shapes}", file=sys.stderr, flush=True)
    # algorithmic bytes per launch with every instance active (padded sizes:
    # each instance's vectors are padded to whole 256-element chunks)
    sv = 8 if precision == "fp64" else 4
    Np = sum((p.n + 255) // 256 * 256 for p in lps)
    Mp = sum((p.m + 255) // 256 * 256 for p in lps)
    alg = {"bk_product<0> (K x')": nnz * (sv + 4) + 4 * (Mp + 1) + sv * Np + sv * Mp,
           "bk_dual (y, K x, q, K x' read; y', K x' written)": 6 * sv * Mp,
           "bk_product<1> (K'y')": nnz * (sv + 4) + 4 * (Np + 1) + sv * Mp + sv * Np,
           "bk_update (averages and next primal)": 11 * sv * Np + 6 * sv * Mp}
    # warm-up: a short solve (graph capture, caches)
    bt.solve(1e-30, 64 * max(args.warmup, 1))
    torch.cuda.synchronize()
    return lps, bt, shapes, alg, nnz, gen_s, load_s


def run_batch(args, precision, seq_sample):
    """The batch's time to rel KKT 1e-4 and the sequential comparison on
    every (count/seq_sample)-th instance, as a dict."""
    import numpy as np
    import torch
    from paper_2312_14832_amd import lp

    lps, bt, shapes, alg, nnz, gen_s, load_s = _batch_setup(args, precision)
    t0 = time.perf_counter()
    bt.solve(1e-4, 10**6, args.ttt_limit)
    torch.cuda.synchronize()
    batch_s = time.perf_counter() - t0
    infos = [bt.info(i) for i in range(len(lps))]
    solved = sum(1 for d in infos if d["status"] == "OPTIMAL")
    iters = np.array([d["iterations"] for d in infos])
    print(f"[bench] batch: {solved}/{len(lps)} optimal in {batch_s:.2f}s; iterations median {np.median(iters):.0f} "
          f"max {iters.max()}", file=sys.stderr, flush=True)
    bt.close()
    stride = max(1, len(lps) // max(seq_sample, 1))
    sample = list(range(0, len(lps), stride))
    seq_s = 0.0
    seq_iters, seq_times = [], []
    for i in sample:
        p = lp.Problem(lps[i], precision=precision, stream=torch.cuda.current_stream())
        p.solve(1e-30, 64)   # same warm-up as the batch
        t1 = time.perf_counter()
        d = p.solve(1e-4, 10**6, args.ttt_limit)
        torch.cuda.synchronize()
        seq_times.append(time.perf_counter() - t1)
        seq_s += seq_times[-1]
        seq_iters.append(d["iterations"])
        p.close()
    seq_est = seq_s * len(lps) / len(sample)
    # the extrapolation's standard error: the sample is every stride-th
    # instance, so its per-instance times are treated as a random sample
    seq_times = np.array(seq_times)
    seq_err = len(lps) * float(np.std(seq_times, ddof=1)) / np.sqrt(len(sample)) if len(sample) > 1 else None
    print(f"[bench] sequential: {len(sample)} instances in {seq_s:.2f}s -> {seq_est:.1f}s for all "
          f"(speedup {seq_est / batch_s:.1f}x)", file=sys.stderr, flush=True)
    out = {
        "metric": "batch time-to-1e-4 KKT",
        "value": len(lps) / batch_s,
        "unit": "LPs/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * batch_s,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if precision == "fp64" else "f32+f64acc",
        "data": "synthetic",
        "config": {"workload": f"batch_{len(lps)}_uneven_lps", "count": len(lps), "sum_nnz": nnz,
                   "row_blocks": {k: {"nnz_per_block": v[0], "rows_per_block": v[1]} for k, v in shapes.items()},
                   "seeds": [1000, 1000 + len(lps) - 1], "precision": precision, "tol": 1e-4},
        "batch_seconds": batch_s,
        "solved": solved,
        "iterations_median": float(np.median(iters)),
        "iterations_max": int(iters.max()),
        "sequential": {"sample": len(sample), "stride": stride, "seconds_sample": seq_s,
                       "seconds_extrapolated": seq_est, "seconds_extrapolated_stderr": seq_err,
                       "speedup": seq_est / batch_s, "iterations_median": float(np.median(seq_iters))},
        "alg_bytes_per_launch": alg,
        "load_s": load_s,
        "gen_s": gen_s,
    }
    return out


def bench_warmstart(args):
    """Learned warm start on the parametric family (fixed K: n=2e5,
    m1=m2=5e4, 10 nonzeros per column; b, h, c from the base certificate
    perturbed by 10% relative noise).  Training labels: this solver (the
    shared-matrix batch, FP64) to rel KKT 1e-5; targets are the scaled
    solution and the log primal weight of each label solve; network 256 ->
    3x1024 ReLU -> 64 -> n+m+1 in BF16 on the GPU.  Held-out members are
    solved (shared batch, iterations) from: cold; the base solution (mean
    label) with the default primal weight, i.e. the method without the
    network; the base solution with the family's primal weight; the
    network's point with the default weight; the network's point and
    weight.  Single-handle wall times (sketch + inference included) are
    taken on a sample of the held-out members.
    """
    import numpy as np
    import torch
    from paper_2312_14832_amd import gen, warmstart as ws

    log = lambda msg: print(f"[bench] {msg}", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    base = gen.parametric_base(4)
    fam = ws.Family(base)
    train_lps = [gen.parametric_instance(base, 10_000 + i) for i in range(args.ws_train)]
    eval_lps = [gen.parametric_instance(base, 30_000 + i) for i in range(args.ws_eval)]
    log(f"generated family n={base.n} m={base.m} nnz={base.nnz}: {len(train_lps)} train, {len(eval_lps)} held out "
        f"in {time.perf_counter() - t0:.1f}s")
    t0 = time.perf_counter()
    Z, infos = ws.solve_labels(train_lps, tol=1e-5, group=128, max_iters=20000, log=log,
                               precision=args.ws_label_precision)
    label_s = time.perf_counter() - t0
    ok = sum(1 for i in infos if i["status"] == "OPTIMAL")
    log(f"labels: {ok}/{len(infos)} optimal at 1e-5 in {label_s:.1f}s ({len(infos) / label_s:.2f} per second)")
    keep = np.array([i["status"] == "OPTIMAL" for i in infos])
    T = fam.encode(Z[keep], [i["omega"] for i, k in zip(infos, keep) if k])
    X = fam.sketch([p for p, k in zip(train_lps, keep) if k])
    Td = torch.from_numpy(T).cuda()
    mu = X.mean(0).cpu().numpy()
    sig = X.std(0).cpu().numpy() + 1e-6
    tbase = T.mean(0)
    xb, yb, om_fam = fam.decode(tbase)
    Xe = fam.sketch(eval_lps)

    def trained(count):
        net = ws.Net(fam.out_dim, max_batch=256)
        net.init_params(0, out_bias=T[:count].mean(0))
        net.set_norm(mu, sig)
        t1 = time.perf_counter()
        losses = ws.train(net, X[:count].contiguous(), Td[:count].contiguous(), epochs=args.ws_epochs, batch=256,
                          lr=1e-3)
        torch.cuda.synchronize()
        pred = np.concatenate([net.forward(Xe[b0:b0 + 256].contiguous()).cpu().numpy()
                               for b0 in range(0, len(eval_lps), 256)])
        return net, losses, time.perf_counter() - t1, pred

    def mean_iters(starts, label):
        t1 = time.perf_counter()
        r = ws.solve_starts(eval_lps, starts, tol=1e-4, group=128)
        it = np.array([t["iterations"] for t in r], np.float64)
        out = {"iters_mean": float(it.mean()), "iters_median": float(np.median(it)),
               "optimal": sum(1 for t in r if t["status"] == "OPTIMAL"), "fallbacks": sum(t["fallback"] for t in r),
               "batch_seconds": time.perf_counter() - t1}
        log(f"{label}: mean {out['iters_mean']:.0f} it, median {out['iters_median']:.0f}, "
            f"{out['optimal']}/{len(r)} optimal, {out['fallbacks']} fallbacks ({out['batch_seconds']:.1f}s)")
        return out

    used = int(keep.sum())
    net, losses, train_s, pred = trained(used)
    starts_net = [fam.decode(r) for r in pred]
    summ = {
        "cold": mean_iters([None] * len(eval_lps), "cold"),
        "base_start": mean_iters([(xb, yb, 0.0)] * len(eval_lps), "base solution, default weight"),
        "base_start_family_omega": mean_iters([(xb, yb, om_fam)] * len(eval_lps),
                                              "base solution, family weight"),
        "net_point_default_omega": mean_iters([(x, y, 0.0) for x, y, _ in starts_net],
                                              "network point, default weight"),
        "net_start": mean_iters(starts_net, "network point and weight"),
    }
    summ["base_start_family_omega"]["omega"] = om_fam
    # learning curve: the network trained on the first `count` labels
    curve = []
    for count in sorted({c for c in (used // 8, used // 4, used // 2, 2048) if 64 <= c < used}):
        _, lc, _, pc = trained(count)
        r = mean_iters([fam.decode(v) for v in pc], f"network trained on {count}")
        curve.append({"train": count, "loss_last": lc[-1], "iters_mean": r["iters_mean"]})
    curve.append({"train": used, "loss_last": losses[-1], "iters_mean": summ["net_start"]["iters_mean"]})
    # single-handle wall time on a sample (sketch and inference in the warm time)
    rows = []
    for i, p in enumerate(eval_lps[:args.ws_time_sample]):
        ic, tc, _ = ws.solve_with_start(p, None)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        out = net.forward(fam.sketch([p]))[0].cpu().numpy()
        x0, y0, om = fam.decode(out)
        inf_s = time.perf_counter() - t1
        iw, tw, fbw = ws.solve_with_start(p, np.concatenate([x0, y0]), omega=om)
        rows.append((ic["iterations"], tc, iw["iterations"], tw + inf_s, fbw, inf_s))
    r = np.array(rows, dtype=np.float64)
    gm = lambda v: float(np.exp(np.mean(np.log(np.maximum(v, 1e-12)))))
    timing = {"sample": len(rows), "cold_time_mean_s": r[:, 1].mean(), "cold_time_geomean_s": gm(r[:, 1]),
              "net_time_mean_s": r[:, 3].mean(), "net_time_geomean_s": gm(r[:, 3]),
              "inference_mean_s": r[:, 5].mean(), "fallbacks": int(r[:, 4].sum()),
              "cold_iters_mean": r[:, 0].mean(), "net_iters_mean": r[:, 2].mean()}
    log(f"single-handle sample of {len(rows)}: cold {timing['cold_time_mean_s']:.3f}s, "
        f"network {timing['net_time_mean_s']:.3f}s (inference {timing['inference_mean_s'] * 1e3:.1f} ms)")
    out = {
        "metric": "time-to-1e-4 KKT, warm-start vs plain",
        "value": timing["cold_time_mean_s"] / timing["net_time_mean_s"],
        "unit": "x speedup (mean cold time / mean warm time, single-handle solves)",
        "n_gpus": 1, "steps": len(eval_lps), "warmup": 0,
        "ms_per_step": 1e3 * timing["net_time_mean_s"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64 solve, bf16 network",
        "data": "synthetic",
        "config": {"workload": "parametric_family_n200000", "n": base.n, "m1": base.m1, "m2": base.m - base.m1,
                   "nnz": base.nnz, "train": len(train_lps), "train_used": used, "held_out": len(eval_lps),
                   "label_tol": 1e-5, "label_precision": args.ws_label_precision, "tol": 1e-4,
                   "epochs": args.ws_epochs, "perturbation": 0.1},
        "summary": summ,
        "learning_curve": curve,
        "timing": timing,
        "training": {"loss_first": losses[0], "loss_last": losses[-1], "seconds": train_s, "label_seconds": label_s,
                     "labels_per_second": len(infos) / label_s},
    }
    print(json.dumps(out))


def shared_bytes(which, n, m, nnz, B, s=8):
    """Algorithmic bytes of one launch of the shared batch's two product
    kernels for B instances: the matrix once (values, int32 columns, row
    pointers), the gathered vector once per instance, and the vectors the
    fused step reads and writes per instance (the single-LP counts times B)."""
    if which == 0:   # sk_dual: K x' + dual step (y, Kx, q read; y', Kx' written)
        return nnz * (s + 4) + 4 * (m + 1) + B * s * n + 5 * B * s * m
    # sk_update: K'y' + averages + next primal (x, c, l, u, xbar, K'ybar read; K'y, xbar, K'ybar, x'' written;
    # y, Kx read and ybar, Kxbar read and written)
    return nnz * (s + 4) + 4 * (n + 1) + B * s * m + 10 * B * s * n + 6 * B * s * m


def bench_shared(args):
    """The shared-matrix batch on `--shared-count` members of the warm-start
    family (n=2e5, m1=m2=5e4, 2e6 nonzeros): a warm-up solve, then a fresh
    solve of `steps` windows of 64 attempt slots timed end to end (start
    products included; instance-iterations per second), and the two product
    kernels' algorithmic bytes per launch."""
    import numpy as np
    import torch
    from paper_2312_14832_amd import gen, lp

    base = gen.parametric_base(4)
    B = args.shared_count
    lps = [gen.parametric_instance(base, 10_000 + i) for i in range(B)]
    sh = lp.Shared(lps, precision=args.precision)
    sh.solve(1e-30, ITERS_PER_STEP * max(args.warmup, 1))   # warm-up (every solve starts afresh)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sh.solve(1e-30, ITERS_PER_STEP * args.steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    its = sum(sh.info(i)["iterations"] for i in range(B))
    s = 8 if args.precision == "fp64" else 4
    out = {"metric": "shared-matrix batch instance-iterations/sec", "value": its / dt, "unit": "instance-it/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * dt / args.steps,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64" if args.precision == "fp64" else "f32+f64acc", "data": "synthetic",
           "config": {"workload": f"parametric_family_n200000_shared{B}", "n": base.n, "m": base.m,
                      "nnz": base.nnz, "instances": B, "precision": args.precision},
           "alg_bytes_per_launch": {"sk_dual": shared_bytes(0, base.n, base.m, base.nnz, B, s),
                                    "sk_update": shared_bytes(1, base.n, base.m, base.nnz, B, s)}}
    print(f"[bench] {B} instances: {its / dt:.0f} instance-it/s, {1e3 * dt / (args.steps * ITERS_PER_STEP):.3f} "
          f"ms per slot", file=sys.stderr, flush=True)
    print(json.dumps(out))


def bench_gather(args):
    """The gather ceiling of the sparse products (lp_gather_probe): 2e7
    gathers, as in one product of the 2e6-column LP, from 8 column slices
    dealt to the XCDs as the products deal them (and from one slice, the
    unsliced case), for slices of 256 KiB to 64 MiB of the gathered vector.
    Patterns: i.i.d. uniform indices (a random sparse matrix), the same
    sorted inside each 2048-index chunk (a row block whose entries were
    ordered by column), and consecutive indices (the coalesced bound)."""
    import numpy as np
    import torch
    from paper_2312_14832_amd import lp

    rng = np.random.Generator(np.random.PCG64(7))
    s = 8 if args.precision == "fp64" else 4
    dt = torch.float64 if args.precision == "fp64" else torch.float32
    count = 20_000_000
    rows = []
    for S, kib in [(8, 256), (8, 1024), (8, 2048), (8, 4096), (8, 8192), (1, 16384), (1, 65536)]:
        slice_len = kib * 1024 // s
        per = count // S
        x = torch.ones(S * slice_len, dtype=dt, device="cuda")
        for pattern in ("random", "sorted2048", "consecutive"):
            if pattern == "consecutive":
                h = np.tile(np.arange(per, dtype=np.int64) % slice_len, S)
            else:
                h = rng.integers(0, slice_len, size=S * per)
                if pattern == "sorted2048":
                    h = h.reshape(S, -1)
                    full = (per // 2048) * 2048
                    h[:, :full] = np.sort(h[:, :full].reshape(S, -1, 2048), axis=2).reshape(S, full)
                    h = h.ravel()
            idx = torch.from_numpy(h.astype(np.int32)).cuda()
            ms = lp.gather_probe(idx, x, S, slice_len, reps=20)
            rate = S * per / (ms * 1e-3) / 1e9
            rows.append({"slices": S, "slice_kib": kib, "pattern": pattern, "ms": ms, "G_gathers_s": rate,
                         "useful_GB_s": rate * s})
            print(f"[bench] S={S} slice {kib} KiB {pattern:12s}: {ms:.3f} ms, {rate:.1f} G gathers/s",
                  file=sys.stderr, flush=True)
            del idx
        del x
    head = next(r for r in rows if r["slices"] == 8 and r["slice_kib"] == 2048 and r["pattern"] == "random")
    out = {"metric": "random gathers per second", "value": head["G_gathers_s"], "unit": "G gathers/s",
           "n_gpus": 1, "steps": 20, "warmup": 1, "ms_per_step": head["ms"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64" if s == 8 else "f32", "data": "synthetic",
           "config": {"workload": "gather_probe_2e7", "gathers": count,
                      "headline": "8 slices of 2 MiB, i.i.d. indices (the 2e6-column LP's K product)"},
           "table": rows}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
