"""Benchmark of the SKIS hot path on one MI355X.

One step = the whole path over one synthetic workload with the graph already in HBM:
build_sketch (preprocessing, roots, persistent sampler, compaction, inverse index), then
estimates for 100 seed sets and a greedy max-cover with k = 100 on the sketch.
value = samples per second over the timed steps (T samples per step).

Prints ONE JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time
import types

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def algorithmic_bytes(T: int, entries: int, probed: int) -> int:
    """Bytes the sampler must move: per sample the root record (20 B) and its result meta
    (size 4 + offset 8 + probed 8 B); per node of R_j its row bounds (8 B) and its staged
    id (4 B); per probed in-edge its (col, w) record (8 B)."""
    return 40 * T + 12 * entries + 8 * probed


# (threads, slots, visited, quads per lane) -> (hash size, items per pass) of the first-tier
# kernel the library compiles for that shape
_TIER0 = {(64, 4, 192, 2): (256, 128), (64, 4, 192, 1): (256, 64), (64, 4, 256, 2): (320, 128),
          (64, 4, 256, 1): (320, 64), (64, 2, 256, 1): (320, 64), (64, 3, 256, 1): (320, 64), (64, 2, 384, 1): (512, 64), (64, 6, 256, 2): (320, 192), (64, 8, 128, 2): (172, 256),
          (64, 8, 192, 2): (256, 256), (64, 8, 192, 1): (256, 256), (64, 8, 256, 2): (344, 256),
          (64, 12, 192, 2): (256, 384), (64, 16, 128, 2): (172, 512), (64, 16, 64, 2): (88, 512),
          (256, 16, 128, 2): (172, 1024), (256, 32, 128, 2): (172, 1024), (256, 16, 256, 2): (344, 1024)}


def random_access_probe(dev, table_log2=33, reps=5):
    """Achievable random-access HBM bandwidth: the library's probe reads 2^26 rows at uniformly
    random positions of an 8 GiB table, far above the last-level caches, for the sampler's two
    random granules, 8-byte row bounds and 32-byte edge quads.  Bytes counted: the rows read.
    Best of `reps`, timed with events on torch's stream (where the probe is launched)."""
    import torch

    from paper_1709_03565_amd import skis
    table = torch.zeros(1 << table_log2, dtype=torch.uint8, device=dev)
    sink = torch.zeros(1, dtype=torch.int32, device=dev)
    reads = 1 << 26
    res = {"probe": "skis_probe_random_read: 2^26 uniformly random rows of an 8 GiB table, bytes of the rows read"}
    for rb in (8, 32):
        best = float("inf")
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            skis.probe_random_read(table, rb, reads, sink)
            e1.record()
            e1.synchronize()
            best = min(best, e0.elapsed_time(e1))
        res["rows_%dB_ms" % rb] = best
        res["rows_%dB_gbs" % rb] = reads * rb / (best * 1e-3) / 1e9
    del table, sink
    torch.cuda.empty_cache()
    return res


def tier0_kernel_name(opts) -> str:
    key = (opts.get("threads_per_block", 64), opts.get("slots_per_block", 4), opts.get("visited_threshold", 192),
           opts.get("quads_per_lane", 1))
    hcap, icap = _TIER0[key]
    return "k_sample<%d, %d, %d, %d, %d, %d, 0>" % (key[0], key[1], key[2], hcap, icap, key[3])


def measured_traffic(kname: str, workload: str):
    """HBM bytes per launch of kname from the committed rocprofv3 counter runs, if they were
    taken on the current sampler source (else None)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
    except ValueError:
        return None
    h = hashlib.sha256()
    for f in ("skis_sample.hip", "skis_device.h"):
        h.update(open(os.path.join(ROOT, "paper_1709_03565_amd", "csrc", f), "rb").read())
    if rec.get("source_sha256") != h.hexdigest():
        return None
    e = rec.get("kernels", {}).get(workload, {}).get(kname)
    return e["hbm_bytes_per_launch"] if e else None


def cpu_baseline(g, wl, sets, k, T):
    import numpy as np

    import oracle
    threads = len(os.sched_getaffinity(0))
    log("cpu baseline: oracle with %d threads" % threads)
    t = time.perf_counter()
    oracle.build_sketch(g.row_ptr, g.col, g.w, seed=1, j0=0, j1=1, nthreads=threads)
    t_fixed = time.perf_counter() - t
    # size the sample for roughly 15 s of sampling
    n0 = 1 << 12
    t = time.perf_counter()
    oracle.build_sketch(g.row_ptr, g.col, g.w, seed=1, j0=0, j1=n0, nthreads=threads)
    rate = n0 / max(time.perf_counter() - t - t_fixed, 1e-3)
    Ns = int(min(max(rate * 15.0, 1 << 14), T))
    Ns = 1 << int(math.log2(Ns))
    t = time.perf_counter()
    sk = oracle.build_sketch(g.row_ptr, g.col, g.w, seed=1, j0=0, j1=Ns, nthreads=threads)
    t_build = time.perf_counter() - t
    _, q = oracle.row_prefix(g.row_ptr, g.w)
    set_ptr, set_nodes = sets
    t = time.perf_counter()
    oracle.inverse(g.n, sk.sample_ptr, sk.nodes)
    oracle.estimate(g.n, sk.sample_ptr, sk.nodes, q, sk.Gamma, set_ptr=set_ptr, set_nodes=set_nodes)
    oracle.greedy(g.n, sk.sample_ptr, sk.nodes, q, sk.Gamma, k)
    t_query = time.perf_counter() - t
    per_sample = max(t_build - t_fixed, 1e-9) / Ns
    t_full = t_fixed + per_sample * T + t_query * (T / Ns)
    log("cpu baseline: Ns=%d build %.2fs (fixed %.2fs) queries %.2fs -> %.3g samples/s" %
        (Ns, t_build, t_fixed, t_query, T / t_full))
    return {
        "value": T / t_full,
        "unit": "samples/s",
        "cores": threads,
        "kind": "oracle",
        "sample": ("oracle (C, %d threads) on sample ids [0, %d) of the same workload: preprocessing "
                   "%.2f s once + %.3g s/sample sampling, plus inverse index, the 100 estimates and greedy "
                   "k=%d on that sketch (%.2f s) scaled by T/%d; extrapolated to T=%d" %
                   (threads, Ns, t_fixed, per_sample, k, t_query, Ns, T)),
        "sampling_only_samples_per_s": 1.0 / per_sample,
    }


def serve(args):
    """Open-loop serving over the resident 4M-node TRI sketch (2^25 samples): Poisson
    arrivals, Zipf(1.5) set sizes in 1..1000, latency from scheduled arrival to the result
    in host memory; the first second is warm-up."""
    import numpy as np
    import torch

    from paper_1709_03565_amd import inputs, skis
    name = "cl4m_tri" if args.workload == "cl1m_wc" else args.workload
    wl = inputs.WORKLOADS[name]
    T = args.samples or wl["T"]
    g = inputs.workload_graph(name)
    log("serve: graph %s n=%d m=%d, T=%d" % (name, g.n, g.m, T))
    torch.cuda.set_device(0)
    rp, col, w = (torch.from_numpy(x).cuda() for x in (g.row_ptr, g.col, g.w))
    sk = skis.build_sketch(rp, col, w, T, inputs.SAMPLE_SEED)
    inf = sk.info()
    warm_s = 1.0
    nq = int(round(args.rate * (warm_s + args.duration)))
    set_ptr, set_nodes, arrival = inputs.serving_trace(g.n, nq, args.rate, seed=11)
    log("serve: %d queries over %.1f s, mean |S| %.2f" % (nq, arrival[-1] / 1e6, set_ptr[-1] / nq))
    srv = skis.Server(sk)
    t = time.perf_counter()
    cov, est, lat = srv.replay(set_ptr, set_nodes, arrival)
    wall = time.perf_counter() - t
    st = srv.stats()
    srv.close()
    meas = arrival >= warm_s * 1e6
    lm = lat[meas]
    t_first = arrival[meas][0]
    t_last_done = np.max(arrival[meas] + lm)
    achieved = meas.sum() / ((t_last_done - t_first) * 1e-6)
    # alone vs mix: the same sets estimated in one plain batch call
    acov, aest = sk.estimate(torch.from_numpy(set_ptr).cuda(), torch.from_numpy(set_nodes).cuda())
    acov = acov.cpu().numpy().astype(np.uint64)
    aest = aest.cpu().numpy()
    same = bool(np.array_equal(acov, cov) and np.array_equal(aest, est))
    # work per query: entries of H(v) walked, sum of deg_H over the set
    node_ptr = sk.inverse()[0].cpu().numpy()
    degH = np.diff(node_ptr)
    work = np.add.reduceat(degH[set_nodes], set_ptr[:-1]) if len(set_nodes) else np.zeros(nq, np.int64)
    wm = work[meas]
    heavy = wm >= np.percentile(wm, 99)
    line = {
        "metric": "SKIS serving latency p99",
        "value": float(np.percentile(lm, 99)),
        "unit": "us",
        "n_gpus": 1,
        "higher_is_better": False,
        "vs_baseline": None,
        "dtype": "u64/f64",
        "data": "synthetic",
        "config": {"workload": "%s: n=%d m=%d, resident sketch of T=%d samples; open-loop Poisson %.0f q/s, "
                               "Zipf(1.5) set sizes in 1..1000, members uniform; %.0f s warm-up + %.0f s measured"
                               % (name, g.n, g.m, T, args.rate, warm_s, args.duration)},
        "p50_us": float(np.percentile(lm, 50)),
        "p90_us": float(np.percentile(lm, 90)),
        "p99_us": float(np.percentile(lm, 99)),
        "p999_us": float(np.percentile(lm, 99.9)),
        "max_us": float(lm.max()),
        "offered_qps": args.rate,
        "achieved_qps": float(achieved),
        "queries_measured": int(meas.sum()),
        "replay_wall_s": wall,
        "batches": st["batches"],
        "mean_batch": st["queries"] / max(st["batches"], 1),
        "max_batch": st["max_batch"],
        "batch_hist_pow2": st["batch_hist"],
        "server_device_bytes": st["device_bytes"],
        "sketch_entries": inf.entries,
        "alone_vs_mix_identical": same,
        "work_entries_p50": float(np.percentile(wm, 50)),
        "work_entries_p99": float(np.percentile(wm, 99)),
        "work_entries_max": int(wm.max()),
        "p50_us_heaviest_1pct": float(np.percentile(lm[heavy], 50)),
        "p99_us_rest": float(np.percentile(lm[~heavy], 99)),
    }
    log("serve: p50 %.1f us p99 %.1f us achieved %.0f q/s, %d batches (mean %.2f), identical alone/mix: %s" %
        (line["p50_us"], line["p99_us"], achieved, st["batches"], line["mean_batch"], same))
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cl1m_wc")
    ap.add_argument("--samples", type=int, default=0, help="override T (default: the workload's)")
    ap.add_argument("--queries", type=int, default=100)
    ap.add_argument("--k", type=int, default=100)
    ap.add_argument("--slots", type=int, default=0)
    ap.add_argument("--visited", type=int, default=0)
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--big-row", type=int, default=0)
    ap.add_argument("--qpl", type=int, default=0, help="edge quads per lane per sweep in the first tier (1 or 2)")
    ap.add_argument("--form", type=int, default=0, help="0: persistent sampler, 1: plain (one launch per level)")
    ap.add_argument("--no-autotune", action="store_true", help="use the library's default sampler shape")
    ap.add_argument("--no-plain-compare", action="store_true",
                    help="skip the untimed plain-form build that is reported beside the persistent sampler")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve", action="store_true",
                    help="serving benchmark instead: open-loop Poisson query stream against a resident sketch")
    ap.add_argument("--rate", type=float, default=50000.0, help="--serve: offered queries per second")
    ap.add_argument("--duration", type=float, default=10.0, help="--serve: measured seconds (after 1 s warm-up)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (for scaling HBM byte counters) and exit")
    args = ap.parse_args()

    if args.calibrate_copy:
        import torch
        nbytes = args.calibrate_copy << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": nbytes, "launches": 3}), flush=True)
        return

    if args.gpus != 1:
        print("bench.py measures one GPU only: the sketch shards by sample id with no communication, "
              "and this benchmark runs and reports a single GPU (got --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1709_03565_amd import inputs, skis

    if args.serve:
        serve(args)
        return

    wl = inputs.WORKLOADS[args.workload]
    T = args.samples or wl["T"]
    build_only = bool(wl.get("build_only"))
    log("workload", args.workload, wl, "T", T)
    t = time.perf_counter()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if wl.get("device_graph"):
        # drawn on the GPU: a host build of this size takes minutes
        rp, col, w = inputs.chung_lu_graph_device(wl["n"], wl["m"], wl["beta"], wl["seed"], wl["model"], dev)
        torch.cuda.synchronize()
        g = types.SimpleNamespace(n=wl["n"], m=wl["m"])
    else:
        g = inputs.workload_graph(args.workload)
        rp = torch.from_numpy(g.row_ptr).to(dev)
        col = torch.from_numpy(g.col).to(dev)
        w = torch.from_numpy(g.w).to(dev)
    log("graph ready in %.1fs: n=%d m=%d" % (time.perf_counter() - t, g.n, g.m))
    if build_only:
        # the build alone is the step: no autotuning sweep, no plain comparison build (the
        # captured form is built once beside it) and no oracle baseline at this size
        args.no_autotune = args.no_plain_compare = args.no_cpu_baseline = True
    sets = inputs.random_sets(g.n, args.queries, 50, seed=7)
    set_ptr_np, set_nodes_np = inputs.sets_to_csr(sets)
    set_ptr = torch.from_numpy(set_ptr_np).to(dev)
    set_nodes = torch.from_numpy(set_nodes_np).to(dev)
    opts = {}
    if args.slots:
        opts["slots_per_block"] = args.slots
    if args.visited:
        opts["visited_threshold"] = args.visited
    if args.threads:
        opts["threads_per_block"] = args.threads
    if args.big_row:
        opts["big_row"] = args.big_row
    if args.qpl:
        opts["quads_per_lane"] = args.qpl
    if args.form:
        opts["form"] = args.form
    tuned = None
    if not args.no_autotune and args.form == 0 and not (args.slots or args.visited or args.threads or args.big_row
                                                         or args.qpl):
        from paper_1709_03565_amd import autotune
        tuned = autotune.autotune(rp, col, w, pilot_samples=T, log=log)
        opts.update(autotune.options_from(tuned))
        log("autotuned options: %s (%.2f ms on the pilot)" % (autotune.options_from(tuned), tuned["ms"]))
    torch.cuda.synchronize()

    def step():
        if build_only:
            sk = skis.build_sketch(rp, col, w, T, inputs.SAMPLE_SEED, build_inverse_index=0, **opts)
            inf = sk.info()
            sk.free()
            return inf, None, None
        sk = skis.build_sketch(rp, col, w, T, inputs.SAMPLE_SEED, **opts)
        sk.estimate(set_ptr, set_nodes)
        seeds, marg, cov, est = sk.greedy(args.k)
        inf = sk.info()
        sk.free()
        return inf, cov, est

    for i in range(args.warmup):
        inf, cov, est = step()
        log("warmup %d: %s" % (i, inf))
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        infos.append(step())
        log("step %d done" % i)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    inf = infos[-1][0]
    ms_step = elapsed * 1000.0 / args.steps
    value = T * args.steps / elapsed
    sampler_ms = sum(x[0].ms_tier0 + x[0].ms_tier1 + x[0].ms_tier2 for x in infos) / len(infos)
    tier0_ms = sum(x[0].ms_tier0 for x in infos) / len(infos)
    b_alg = algorithmic_bytes(T, inf.entries, inf.probed_total)
    # the dominant kernel is the first sampler tier: one launch per step, timed with HIP
    # events on its stream; its algorithmic bytes are those of the samples it finishes
    b_alg0 = algorithmic_bytes(inf.tier_samples[0], inf.tier_entries[0], inf.tier_probed[0])
    achieved = b_alg0 / (tier0_ms * 1e-3) / 1e9
    kname = tier0_kernel_name(opts)
    traffic = measured_traffic(kname, args.workload)
    stages = {k: round(sum(getattr(x[0], k) for x in infos) / len(infos), 3) for k in
              ["ms_preprocess", "ms_roots", "ms_sample", "ms_tier0", "ms_tier1", "ms_tier2", "ms_compact", "ms_inverse"]}
    line = {
        "metric": "SKIS samples/s",
        "value": value,
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64/f64",
        "data": "synthetic",
        "config": {
            "workload": "%s: directed Chung-Lu n=%d m=%d beta=%g, %s weights fp32, T=%d IIS samples, Philox seed %d; "
                        % (args.workload, g.n, g.m, wl["beta"], wl["model"].upper(), T, inputs.SAMPLE_SEED)
                        + ("graph drawn on the GPU; step = build_sketch without the inverse index" if build_only else
                           "step = build_sketch + inverse index + %d estimates (|S| 1-50) + greedy k=%d"
                           % (args.queries, args.k)),
            "T": T, "n": g.n, "m": g.m,
        },
        "edges_probed_per_s": inf.probed_total * args.steps / elapsed,
        "sampler_samples_per_s": T / (sampler_ms * 1e-3),
        "entries": inf.entries,
        "probed_total": inf.probed_total,
        "deferred": inf.deferred,
        "deferred_global": inf.deferred_global,
        "stages_ms": stages,
        "roofline": {
            "bound": "hbm",
            "kernel": kname,
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "alg_bytes_per_launch": b_alg0,
            "launch_ms": tier0_ms,
            "tier0_samples": inf.tier_samples[0],
            "tier0_entries": inf.tier_entries[0],
            "tier0_probed": inf.tier_probed[0],
            "chain_alg_bytes": b_alg,
            "chain_ms": sampler_ms,
            "chain_gbs": b_alg / (sampler_ms * 1e-3) / 1e9,
        },
    }
    if tuned is not None:
        line["config"]["sampler_options"] = autotune.options_from(tuned)
    if not args.no_plain_compare and args.form == 0:
        sk = skis.build_sketch(rp, col, w, T, inputs.SAMPLE_SEED, form=1, build_inverse_index=0)
        pinf = sk.info()
        sk.free()
        line["plain_form"] = {"sampler_ms": pinf.ms_tier0, "levels": pinf.plain_levels,
                              "persistent_sampler_ms": sampler_ms,
                              "speedup_persistent_over_plain": pinf.ms_tier0 / sampler_ms}
        log("plain form: sampler %.1f ms over %d level launches; persistent %.1f ms" %
            (pinf.ms_tier0, pinf.plain_levels, sampler_ms))
    if (build_only or not args.no_plain_compare) and args.form == 0:
        # the captured form: the same chain captured into a HIP graph, replayed per chunk
        cinfs = []
        for _ in range(1 if build_only else 2):
            sk = skis.build_sketch(rp, col, w, T, inputs.SAMPLE_SEED, form=2, build_inverse_index=0,
                                   **{k: v for k, v in opts.items() if k != "form"})
            cinfs.append(sk.info())
            sk.free()
        cinf = min(cinfs, key=lambda x: x.ms_tier0)
        line["captured_form"] = {"sampler_ms": cinf.ms_tier0, "graph_replays": cinf.graph_replays,
                                 "chunk_samples": -(-T // cinf.graph_replays),
                                 "persistent_sampler_ms": sampler_ms}
        log("captured form: sampler %.1f ms over %d graph replays; persistent %.1f ms" %
            (cinf.ms_tier0, cinf.graph_replays, sampler_ms))
    # the tier-0 launch's algorithmic bandwidth against what random 32-byte reads reach
    try:
        ra = random_access_probe(dev)
        ra["tier0_frac_of_32B"] = achieved / ra["rows_32B_gbs"]
        log("random-access probe: %.0f GB/s in 8-B rows, %.0f GB/s in 32-B rows; tier 0 at %.2f of the latter" %
            (ra["rows_8B_gbs"], ra["rows_32B_gbs"], ra["tier0_frac_of_32B"]))
    except Exception as ex:  # a measurement aid: its failure does not void the step's numbers
        ra = {"error": str(ex).splitlines()[0]}
        log("random-access probe failed:", ra["error"])
    line["random_access"] = ra
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(g, wl, (set_ptr_np, set_nodes_np), args.k, T)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
