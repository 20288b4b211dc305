"""Throughput benchmark of the Direct search on one MI355X.

Workload: the N sweep in single and double precision (N in {16, 256, 4096,
65536, 2^20, 2^21}; X built from cumulative U(0.5, 1.5) gaps scaled to [0, 1];
M = 2^26 uniform queries per (N, dtype)).  One timed step searches every
(N, dtype) case once with the Direct method (subtraction form), inputs already
resident in HBM; the tables are built before timing, as the paper's harness
sets each algorithm up before its clock starts (Sec. 6.1, algorithm TestHarness).

Output: first the detail lines (one JSON object each, key "detail": the
per-case figures, the other layouts and methods, the uses, the learned and the
batched workloads), then, as the LAST line, one compact JSON object (under
1.5 KB): Gqueries/s over the step, the roofline of the dominant search kernel
(timed with HIP events on the launch stream), the CPU oracle timed on a bounded
sample, and the ratios the targets are stated in.  --detail-json PATH also
writes every detail object into one JSON file.
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

HBM_PEAK_GBS = 8000.0  # MI355X published HBM3E bandwidth
# L2 request ceiling: 8 XCDs x 16 L2 channels, each serving one (up to 128-byte) request per
# clock, at 2.4 GHz (39.3 TB/s in 128-byte lines)
L2_PEAK_GREQ_S = 8 * 16 * 2.4
STAGE_NAMES = {1: "PLAIN-LDS", 2: "PLAIN-L2", 3: "RANKCODE-LDS", 4: "PAIRS-L2", 5: "RANKCODE-L2",
               6: "NIBBLE-L2", 7: "NIBBLE-LDS", 8: "GAPCODE-LDS"}


# the sources of the sweep's search kernels and of the tables they read: the counter
# summaries stay valid exactly while these are unchanged
TRAFFIC_SOURCES = ("paper_1506_08620_amd/csrc/ds_search.hip", "paper_1506_08620_amd/csrc/ds_build.hip",
                   "paper_1506_08620_amd/csrc/ds_ops.h", "paper_1506_08620_amd/csrc/ds_internal.h")


def traffic_sources_sha256() -> str:
    import hashlib

    h = hashlib.sha256()
    for p in TRAFFIC_SOURCES:
        h.update(open(os.path.join(ROOT, p), "rb").read())
    return h.hexdigest()


def log(msg: str):
    """A progress line on stderr (the result lines go to stdout)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def measured_traffic(dtype: str, ns, stage_name: str):
    """HBM bytes per launch of the given sweep cases from the committed rocprofv3 counter
    summary, or None when the kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "direct_sweep_hbm_traffic.txt")
    if not os.path.exists(path):
        return None
    vals, cases = {}, {}
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        f = line.split()
        if f[0] == "case":
            cases[(f[1], int(f[2]))] = (float(f[4]), float(f[6]))
        else:
            vals[f[0]] = f[1]
    if vals.get("source_sha256") != traffic_sources_sha256():
        return None
    fs, ws = float(vals["fetch_scale"]), float(vals["write_scale"])
    got = [cases[(dtype, n)] for n in ns if (dtype, n) in cases]
    if not got or len(got) != len(ns):
        return None
    return sum((f * fs + w * ws) * 1024.0 for f, w in got) / len(got)


def measured_l2(dtype: str, ns):
    """L2 requests, hits and misses per launch of the given sweep cases from the committed
    rocprofv3 counter summary (TCC_REQ_sum, TCC_HIT_sum, TCC_MISS_sum), or None when the
    kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "direct_sweep_l2_counters.txt")
    if not os.path.exists(path):
        return None
    vals, cases = {}, {}
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        f = line.split()
        if f[0] == "case":
            cases[(f[1], int(f[2]))] = (float(f[4]), float(f[6]), float(f[8]))
        else:
            vals[f[0]] = f[1]
    if vals.get("source_sha256") != traffic_sources_sha256():
        return None
    got = [cases[(dtype, n)] for n in ns if (dtype, n) in cases]
    if not got or len(got) != len(ns):
        return None
    return tuple(sum(g[i] for g in got) / len(got) for i in range(3))


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--cpu-sample", type=int, default=1 << 22, help="queries per case for the CPU oracle")
    p.add_argument("--no-extras", action="store_true", help="skip the per-method comparison runs")
    p.add_argument("--sizes", type=str, default="", help="comma-separated subset of N (testing)")
    p.add_argument("--m", type=int, default=0, help="queries per case (default 2^26)")
    p.add_argument("--no-batched", action="store_true", help="skip the 10,000-array batched workload")
    p.add_argument("--no-learned", action="store_true", help="skip the learned method on the clustered array")
    p.add_argument("--detail-json", type=str, default="", help="also write the detail objects to this file")
    p.add_argument("--calibrate-copy", action="store_true",
                   help="first run a plain device copy of 2^26 int32 (256 MiB read + 256 MiB written), the "
                        "reference for scaling hardware traffic counters")
    return p.parse_args()


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark measures one GPU; run with --gpus 1 "
                                   "(the queries of a search shard across GPUs with no exchange; each GPU runs this measurement on its share)"}))
        sys.exit(2)

    import torch

    import paper_1506_08620_amd as ds
    import workloads as W

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.calibrate_copy:
        src = torch.ones(1 << 26, dtype=torch.int32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    M = args.m or W.SWEEP_M
    sizes = [int(s) for s in args.sizes.split(",")] if args.sizes else list(W.SWEEP_N)
    cases = []
    # the first build in the process also loads the library's code objects: not timed
    ds.build(torch.from_numpy(W.sweep_array(16, np.float32)).to(dev)).destroy()
    for dt in (np.float32, np.float64):
        for n in sizes:
            X = W.sweep_array(n, dt)
            x_d = torch.from_numpy(X).to(dev)
            z_d = W.sweep_queries_torch(M, dt, dev)
            out = torch.empty(M, dtype=torch.int32, device=dev)
            torch.cuda.synchronize()
            times = []
            for r in range(5):  # the median of five builds; the last one is kept
                t0 = time.perf_counter()
                idx = ds.build(x_d)
                torch.cuda.synchronize()
                times.append(time.perf_counter() - t0)
                if r < 4:
                    idx.destroy()
            cases.append(dict(n=n, dt=dt, X=X, x=x_d, z=z_d, out=out, idx=idx, build_s=float(np.median(times))))

    stream = torch.cuda.current_stream()
    log(f"sweep: {len(cases)} cases built")

    def step(ev=None):
        for k, c in enumerate(cases):
            if ev is not None:
                ev[k][0].record(stream)
            ds.search(c["idx"], c["z"], out=c["out"], stream=stream)
            if ev is not None:
                ev[k][1].record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # timed region: exactly K steps between synchronisations
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    # per-launch kernel times with HIP events on the launch stream (separate pass)
    # (steps back to back, as in the timed region, so that no case starts on an idle GPU)
    per = [[] for _ in cases]
    evs = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in cases]
           for _ in range(args.steps)]
    for ev in evs:
        step(ev)
    torch.cuda.synchronize()
    for ev in evs:
        for k, (a, b) in enumerate(ev):
            per[k].append(a.elapsed_time(b))

    total_q = M * len(cases) * args.steps
    value = total_q / wall / 1e9
    case_rows = []
    groups = {}
    for k, c in enumerate(cases):
        ms = float(np.mean(per[k]))
        ms_med, ms_min = float(np.median(per[k])), float(np.min(per[k]))
        S = np.dtype(c["dt"]).itemsize
        bytes_per_launch = M * (S + 4)
        inf = c["idx"].info()
        dts = "f32" if S == 4 else "f64"
        row = dict(N=c["n"], dtype=dts, gq_s=round(M / ms / 1e6, 2),
                   gq_s_median=round(M / ms_med / 1e6, 2), gq_s_best=round(M / ms_min / 1e6, 2),
                   gbs=round(bytes_per_launch / ms / 1e6, 1), hbm_frac=round(bytes_per_launch / ms / 1e6 / HBM_PEAK_GBS, 4),
                   kernel_ms=round(ms, 5), kernel_ms_median=round(ms_med, 5), kernel_ms_min=round(ms_min, 5),
                   layout=STAGE_NAMES[inf["staged"]], R=inf["R"],
                   table_bytes=inf["table_bytes"], build_ns_per_elem=round(c["build_s"] * 1e9 / (c["n"] + 1), 2))
        # HBM bytes this case's launch moved by the committed counters (FETCH_SIZE + WRITE_SIZE)
        hbm = measured_traffic(dts, [c["n"]], row["layout"])
        row["measured_hbm_bytes"] = None if hbm is None else int(hbm)
        row["measured_hbm_gbs"] = None if hbm is None else round(hbm / ms / 1e6, 1)
        case_rows.append(row)
        key = (row["dtype"], row["layout"])
        g = groups.setdefault(key, [0.0, 0, 0, []])
        g[0] += ms
        g[1] += 1
        g[2] += bytes_per_launch
        g[3].append(c["n"])
    dom_key = max(groups, key=lambda k: groups[k][0])
    g = groups[dom_key]
    avg_ms = g[0] / g[1]
    avg_bytes = g[2] / g[1]
    achieved = avg_bytes / avg_ms / 1e6
    kernel_name = "direct_search_kernel<{},SUB,{}>".format("float" if dom_key[0] == "f32" else "double", dom_key[1])
    traffic = measured_traffic(dom_key[0], g[3], dom_key[1])
    roofline = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4), traffic=None if traffic is None else int(traffic),
                    kernel=kernel_name, cases=[f"{dom_key[0]} N={n}" for n in g[3]],
                    launches_per_step=g[1], bytes_per_launch=int(avg_bytes), avg_launch_ms=round(avg_ms, 5),
                    traffic_over_algorithmic=None if traffic is None else round(traffic / avg_bytes, 3))
    # the second ceiling of the tables read through L2: requests per second against the L2's
    # request rate, from the committed counters of the same launches
    l2 = measured_l2(dom_key[0], g[3])
    if l2 is not None:
        req, hit, miss = l2
        roofline["l2"] = dict(req_per_launch=int(req), achieved_greq_s=round(req / avg_ms / 1e6, 1),
                              peak_greq_s=L2_PEAK_GREQ_S, frac=round(req / avg_ms / 1e6 / L2_PEAK_GREQ_S, 4),
                              hit_rate=round(hit / req, 4), req_per_query=round(req / M, 3))

    log(f"sweep: {args.steps} timed steps, {value:.1f} Gq/s")
    # CPU oracle on a bounded sample of the same workload
    cpu = None
    parity = True
    try:
        import oracle

        threads = len(os.sched_getaffinity(0))
        sample = min(args.cpu_sample, M)
        cpu_t = 0.0
        for c in cases:
            zs = c["z"][:sample].cpu().numpy()
            t1 = time.perf_counter()
            ref = oracle.search(c["X"], zs, nthreads=threads)
            cpu_t += time.perf_counter() - t1
            got = c["out"][:sample].cpu().numpy()
            parity = parity and bool(np.array_equal(got, ref))
        cpu = dict(value=round(sample * len(cases) / cpu_t / 1e9, 4), unit="Gqueries/s", cores=threads,
                   kind="oracle", sample=f"first {sample} queries of each of the {len(cases)} (N, dtype) cases, "
                                          f"classic binary search")
        # one core, as the paper's single-core Classic figures
        sample1 = max(1, sample // 16)
        cpu_t1 = 0.0
        for c in cases:
            zs = c["z"][:sample1].cpu().numpy()
            t1 = time.perf_counter()
            oracle.search(c["X"], zs, nthreads=1)
            cpu_t1 += time.perf_counter() - t1
        cpu1 = dict(value=round(sample1 * len(cases) / cpu_t1 / 1e9, 4), unit="Gqueries/s", cores=1, kind="oracle",
                    sample=f"first {sample1} queries of each of the {len(cases)} cases, classic binary search, "
                           f"1 thread")
    except Exception as e:  # the CPU leg must not hide the GPU figure
        cpu = dict(value=None, unit="Gqueries/s", cores=0, kind="oracle", sample=f"failed: {e}")
        cpu1 = None

    log("cpu baseline done")
    extras = {}
    if not args.no_extras:
        extras = compare_methods(ds, cases, M, stream, reps=max(3, min(args.steps, 10)))
        log("other layouts and methods done")
        extras["uses"] = bench_uses(ds, cases, M, stream, reps=max(3, min(args.steps, 10)))
        log("uses done")
    direct_f64_2p20 = next((r["gq_s"] for r in case_rows if r["N"] == 1 << 20 and r["dtype"] == "f64"), None)
    n_cases = len(cases)
    for c in cases:  # free the sweep's buffers first
        c["idx"].destroy()
    cases.clear()
    torch.cuda.empty_cache()
    if not args.no_learned:
        extras["learned_f64_clustered"] = bench_learned(ds, W, dev, stream, reps=10, direct_ref=direct_f64_2p20)
        log("learned done")
    if not args.no_batched:
        extras["batched_f32"] = bench_batched(ds, W, dev, stream, reps=3)
        log("batched done")
        extras["batched_learned_f64_mixture"] = bench_batched_learned(ds, W, dev, stream, reps=5)
        log("batched learned done")

    detail = {"cases": case_rows, "roofline_detail": roofline, "cpu_baseline_detail": cpu,
              "cpu_baseline_1thread_detail": cpu1, **extras}
    if args.detail_json:
        with open(args.detail_json, "w") as f:
            json.dump(detail, f, indent=1)
    for k, v in detail.items():  # one line per object, each well under the 8 KB a log tail keeps
        print(json.dumps({"detail": k, "value": v}))

    # the targets, as ratios
    def min_frac(dts):
        fr = [r["hbm_frac"] for r in case_rows if r["dtype"] == dts and r["N"] <= 1 << 16]
        return min(fr) if fr else None

    targets = {"direct_min_hbm_frac_n_le_2p16": {"f32": min_frac("f32"), "f64": min_frac("f64"), "goal": 0.6}}
    le = extras.get("learned_f64_clustered")
    if le:
        targets["learned_vs_direct_f64_2p20"] = {"ratio": le.get("learned_vs_direct"), "goal": 0.5,
                                                 "learned_gq_s": le["learned"]["gq_s"],
                                                 "no_network_gq_s": le["learned_no_network"]["gq_s"],
                                                 "model_vs_table": float("%.3g" % le["model_vs_direct_table"])}
    bf = extras.get("batched_f32")
    if bf:
        targets["batched_f32_gq_s"] = {"graph": bf["gq_s_graph_replay"], "eager": bf["gq_s_end_to_end"]}
    bl = extras.get("batched_learned_f64_mixture")
    if bl:
        targets["batched_learned_f64_gq_s"] = {"trained": bl["gq_s_end_to_end"],
                                               "no_network": bl["no_network"]["gq_s_end_to_end"]}
    keep = ("bound", "achieved", "peak", "unit", "frac", "traffic", "kernel", "avg_launch_ms", "bytes_per_launch",
            "l2")
    line = {
        "metric": "Gqueries/s and %HBM peak: Direct vs learned vs binary search, FP32/FP64",
        "value": round(value, 2),
        "unit": "Gqueries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"direct-sweep N={sizes} f32+f64, U(0.5,1.5) gaps scaled to [0,1], "
                               f"M={M} uniform queries per case",
                   "queries_per_step": M * n_cases},
        "roofline": {k: roofline[k] for k in keep if k in roofline},
        "cpu_baseline": cpu,
        "cpu_baseline_1thread": None if cpu1 is None else {k: cpu1[k] for k in ("value", "unit", "cores")},
        "parity_sample_bit_exact": parity,
        "targets": targets,
    }
    text = json.dumps(line, separators=(",", ":"))
    if len(text) > 1500:  # never let the headline outgrow what a log tail keeps
        line.pop("targets")
        text = json.dumps(line, separators=(",", ":"))
    print(text)


def compare_methods(ds, cases, M, stream, reps):
    """Other layouts, Direct-FMA and the branch-free binary search on the same inputs (not in the timed step)."""
    import torch

    def timed(idx, c, out):
        ds.search(idx, c["z"], out=out, stream=stream)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            ds.search(idx, c["z"], out=out, stream=stream)
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    res = {"direct_layouts": [], "direct_fma": [], "direct_gap2": [], "direct_gap4": [], "bsearch_leadbit": [],
           "bsearch_eytzinger": []}
    for c in cases:
        S = np.dtype(c["dt"]).itemsize
        tag = dict(N=c["n"], dtype="f32" if S == 4 else "f64")
        out = torch.empty_like(c["out"])
        idx = ds.build(c["x"], layouts=("rankcode", "pairs", "nibble"))
        inf = idx.info()
        lay = {}
        for stage, name in STAGE_NAMES.items():
            try:
                idx.set_tune(stage=stage)
            except ds.DsError:
                continue
            ms = timed(idx, c, out)
            lay[name] = dict(gq_s=round(M / ms / 1e6, 2), same_as_direct=bool(torch.equal(out, c["out"])))
        res["direct_layouts"].append(dict(**tag, layouts=lay, rankcode_bytes=inf["rankcode_bytes"],
                                          pairs_bytes=inf["pairs_bytes"], nibble_bytes=inf["nibble_bytes"]))
        idx.destroy()
        for key, kw in (("direct_fma", dict(form="fma")), ("direct_gap2", dict(method="direct_gap", gap_q=2)),
                        ("direct_gap4", dict(method="direct_gap", gap_q=4)), ("bsearch_leadbit", dict(method="leadbit")),
                        ("bsearch_eytzinger", dict(method="eytzinger"))):
            idx = ds.build(c["x"], **kw)
            inf = idx.info()
            ms = timed(idx, c, out)
            res[key].append(dict(**tag, gq_s=round(M / ms / 1e6, 2),
                                 hbm_frac=round(M * (S + 4) / ms / 1e6 / HBM_PEAK_GBS, 4),
                                 layout=STAGE_NAMES.get(inf["staged"], "?"), table_bytes=inf["table_bytes"],
                                 same_as_direct=bool(torch.equal(out, c["out"]))))
            idx.destroy()
        del out
    return res


def bench_uses(ds, cases, M, stream, reps):
    """The uses of Sec. 2 on the sweep's arrays and queries: the fused histogram and
    interpolation kernels against the same results built from ds_search plus torch ops
    (not in the timed step)."""
    import torch

    def timed(fn):
        fn()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    rows = []
    with torch.cuda.stream(stream):
        for c in cases:
            n, z, idx = c["n"], c["z"], c["idx"]
            S = np.dtype(c["dt"]).itemsize
            counts = torch.zeros(n + 2, dtype=torch.int64, device=z.device)
            out = torch.empty_like(c["out"])
            X = c["x"]
            Y = torch.cumsum(torch.ones(n + 1, dtype=X.dtype, device=X.device), 0)
            y = torch.empty_like(z)

            def hist_fused():
                counts.zero_()
                idx.histogram(z, counts, stream=stream)

            def hist_unfused():
                ds.search(idx, z, out=out, stream=stream)
                return torch.bincount(out.long() + 1, minlength=n + 2)

            def interp_fused():
                idx.interp_linear(Y, z, out=y, stream=stream)

            def interp_unfused():
                ds.search(idx, z, out=out, stream=stream)
                i = out.long().clamp(0, n - 1)
                x0, x1, y0, y1 = X[i], X[i + 1], Y[i], Y[i + 1]
                r = y0 + ((z - x0) / (x1 - x0)) * (y1 - y0)
                r = torch.where(out < 0, Y[0], torch.where(out >= n, Y[n], r))
                return r

            ms = {k: timed(f) for k, f in (("hist_fused", hist_fused), ("hist_unfused", hist_unfused),
                                           ("interp_fused", interp_fused), ("interp_unfused", interp_unfused))}
            hist_fused()
            same_hist = bool(torch.equal(counts, hist_unfused()))
            interp_fused()
            rel = float(((y - interp_unfused()).abs().max() / Y.abs().max()).item())
            rows.append(dict(N=n, dtype="f32" if S == 4 else "f64", layout=STAGE_NAMES[idx.info()["staged"]],
                             **{f"{k}_gq_s": round(M / v / 1e6, 2) for k, v in ms.items()},
                             hist_same_as_unfused=same_hist, interp_max_rel_diff_vs_unfused=rel))
            del counts, out, Y, y
    return rows


def bench_learned(ds, W, dev, stream, reps, direct_ref):
    """Clustered f64 array (N + 1 = 2^20 lognormal draws), 2^26 queries: the learned
    method (trained router), its ablation without the network, and the leading-bit
    binary search on the same inputs.  Direct is infeasible on this array."""
    import torch

    X = W.clustered_array()
    z = W.clustered_queries(X, 1 << 26)
    x_d = torch.from_numpy(X).to(dev)
    z_d = torch.from_numpy(z).to(dev)
    out = torch.empty(z.size, dtype=torch.int32, device=dev)
    M = z.size
    res = {"N": X.size - 1, "M": M, "direct_table_bytes_needed": None}
    gaps = np.diff(X)
    res["direct_table_bytes_needed"] = float(4.0 * (X[-1] - X[0]) / gaps.min())
    ref_out = None
    for name, kw in (("learned", dict(method="learned")),
                     ("learned_eval_fp16_router", dict(method="learned", learn_router="fp16")),
                     ("learned_eval_fp32_router", dict(method="learned", learn_router="fp32")),
                     ("learned_no_network", dict(method="learned", learn_epochs=-1)),
                     ("bsearch_leadbit", dict(method="leadbit"))):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        idx = ds.build(x_d, **kw)
        torch.cuda.synchronize()
        build_s = time.perf_counter() - t0
        for _ in range(reps):  # warm-up long enough for the clocks to settle after the build
            ds.search(idx, z_d, out=out, stream=stream)
        a, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            ds.search(idx, z_d, out=out, stream=stream)
        e.record(stream)
        torch.cuda.synchronize()
        ms = a.elapsed_time(e) / reps
        inf = idx.info()
        row = dict(gq_s=round(M / ms / 1e6, 2), hbm_frac=round(M * 12 / ms / 1e6 / HBM_PEAK_GBS, 4),
                   build_s=round(build_s, 3))
        if name.startswith("learned"):
            _, fb = idx.learned_model()
            row.update(model_bytes=inf["model_bytes"], max_err=inf["max_err"],
                       mean_log2_window=round(inf["mean_log2_window"], 3), fallbacks=fb)
        if ref_out is None:
            ref_out = out.clone()
        else:
            row["same_as_learned"] = bool(torch.equal(out, ref_out))
        res[name] = row
        idx.destroy()
    if direct_ref:
        res["direct_f64_n2p20_sweep_gq_s"] = direct_ref
        res["learned_vs_direct"] = round(res["learned"]["gq_s"] / direct_ref, 3)
    res["model_vs_direct_table"] = res["learned"]["model_bytes"] / res["direct_table_bytes_needed"]
    del z_d, out, ref_out
    torch.cuda.empty_cache()
    return res


def bench_batched(ds, W, dev, stream, reps):
    """10,000 f32 arrays, N_k log-uniform in [8, 65536], M_k = 64 N_k: one ds_search_batched
    call (device build of every array + search), timed end to end with HIP events."""
    import torch

    b = W.batched_f32(with_queries=False)
    z = W.batched_queries_torch(b, dev)
    bt = ds.Batch(torch.from_numpy(b.x_off).to(dev), torch.from_numpy(b.X).to(dev),
                  torch.from_numpy(b.q_off).to(dev), z)
    shape = bt.autotune(stream)
    torch.cuda.synchronize()
    a, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(reps):
        bt.run(stream)
    e.record(stream)
    torch.cuda.synchronize()
    ms = a.elapsed_time(e) / reps
    # the same build + search captured once in a HIP graph with the autotuned shape, timed over replays
    side = torch.cuda.Stream()
    side.wait_stream(stream)
    with torch.cuda.stream(side):
        bt.run()
    stream.wait_stream(side)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        bt.run()
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        g.replay()
        a.record(stream)
        for _ in range(reps):
            g.replay()
        e.record(stream)
    torch.cuda.synchronize()
    ms_graph = a.elapsed_time(e) / reps
    total_q = int(b.q_off[-1])
    meth, _ = bt.report()
    res = dict(arrays=b.num_arrays, total_x=int(b.x_off[-1]), total_q=total_q,
               ms_graph_replay=round(ms_graph, 3), gq_s_graph_replay=round(total_q / ms_graph / 1e6, 2),
               ms_end_to_end=round(ms, 3), gq_s_end_to_end=round(total_q / ms / 1e6, 2),
               hbm_frac_streaming=round(total_q * 8 / ms_graph / 1e6 / HBM_PEAK_GBS, 4),
               direct_arrays=int((meth == ds.METHOD_DIRECT).sum()), autotuned_shape=shape)
    del g, z, bt
    torch.cuda.empty_cache()
    return res


def bench_batched_learned(ds, W, dev, stream, reps):
    """256 f64 mixture arrays (N_k log-uniform in [2^14, 2^20]), 2^28 queries: one
    ds_search_batched call = device build of every array, training of the learned
    arrays' models (all together), routing, fits and search; Direct where its table
    fits under 64 MB.  Timed end to end with HIP events."""
    import torch

    b = W.batched_mixture(with_queries=False)
    z = W.batched_mixture_queries_torch(b, dev)
    x_off, X, q_off = (torch.from_numpy(a).to(dev) for a in (b.x_off, b.X, b.q_off))
    total_q = int(b.q_off[-1])
    res = dict(arrays=b.num_arrays, total_x=int(b.x_off[-1]), total_q=total_q,
               note="end to end: device build, training of every learned model (2 steps, one launch), "
                    "router compilation, fits and search")
    ref = None
    # the trained routers, and the same models with the router replaced by the feature (no network)
    for name, steps in (("trained", 0), ("no_network", -1)):
        bt = ds.Batch(x_off, X, q_off, z, learn_segments=2048, learn_steps=steps, direct_cap_bytes=64 << 20)
        for _ in range(2):
            bt.run(stream)
        torch.cuda.synchronize()
        a, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            bt.run(stream)
        e.record(stream)
        torch.cuda.synchronize()
        ms = a.elapsed_time(e) / reps
        meth, _ = bt.report()
        row = dict(ms_end_to_end=round(ms, 3), gq_s_end_to_end=round(total_q / ms / 1e6, 2),
                   direct_arrays=int((meth == ds.METHOD_DIRECT).sum()),
                   learned_arrays=int((meth == ds.METHOD_LEARNED).sum()), fallbacks=bt.fallbacks())
        if ref is None:
            ref = bt.out.clone()
            res.update(row)
        else:
            row["same_as_trained"] = bool(torch.equal(bt.out, ref))
            res[name] = row
        del bt
    del z, ref
    torch.cuda.empty_cache()
    return res


if __name__ == "__main__":
    main()
