"""Benchmark of the SKIS hot path on one MI355X.

Headline (default workload cl40m_wc: 40M nodes, 1.4B edges, WC, T = 2^26, the largest
configuration that fits one GPU): one step = build_sketch of the whole sketch with the graph
already in HBM (preprocessing, roots, the persistent sampler, compaction; the inverse index is
not built at this size).  value = samples per second over the timed steps (T samples a step).
With --workload cl1m_wc or cl4m_tri a step is the whole path: build_sketch with the inverse
index, 100 estimates and a greedy k = 100.

Beside the headline the same JSON line carries (unless --no-extras): the full steps of the
1M-node WC and 4M-node TRI workloads, a short open-loop serving run over the TRI sketch
(p50/p99 latency, achieved queries/s, alone-vs-mix identity), the build of the same 40M-node
graph with linear threshold weights and the LT sampler (Sec. 6), and the random-read probe at
8, 32, 64 and 128-byte rows.

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


def sample_bytes(T: int, entries: int, probed: int) -> int:
    """Bytes the sampler must move for whole samples: per sample the root record (20 B) and
    its result meta (size 4 + offset 8 + probed 8 B); per node of R_j its row bounds (8 B) and
    its staged id (4 B); per probed in-edge its (col, coin threshold) record (8 B)."""
    return 40 * T + 12 * entries + 8 * probed


def launch_bytes(inf, t: int, lt: bool = False) -> int:
    """Bytes one sampler tier's launch must move for the work it did: the root record and
    result meta of every sample it finished (40 B) and their staged ids (4 B a node), the row
    bounds of every node it expanded (8 B) and the record of every in-edge it swept (8 B).
    A sample resumed from an earlier tier is charged only for what this launch expanded.
    Linear threshold kernels (lt): per sample the alias entry (16 B), the root's row bounds
    (8 B), q (8 B), one running sum (8 B), the picked id (4 B) and the result meta (36 B); per
    further node of R_j its row bounds, one running sum and the picked id (20 B); per node its
    staged id (4 B): 60 B a sample + 24 B a node."""
    if lt:
        return 60 * inf.tier_samples[t] + 24 * inf.tier_entries[t]
    return 40 * inf.tier_samples[t] + 4 * inf.tier_entries[t] + 8 * inf.tier_items[t] + 8 * inf.tier_swept[t]


# (threads, slots, visited, quads per lane) -> (hash size, items per pass) of the first-tier
# kernel the library compiles for that shape
_TIER0 = {(64, 4, 192, 2): (256, 128), (64, 4, 192, 1): (256, 64), (64, 4, 256, 2): (320, 128),
          (64, 4, 256, 1): (320, 64), (64, 2, 256, 1): (320, 64), (64, 3, 256, 1): (320, 64), (64, 2, 384, 1): (512, 64), (64, 6, 256, 2): (320, 192), (64, 8, 128, 2): (172, 256),
          (64, 8, 192, 2): (256, 256), (64, 8, 192, 1): (256, 256), (64, 8, 256, 2): (344, 256),
          (64, 12, 192, 2): (256, 384), (64, 16, 128, 2): (172, 512), (64, 16, 64, 2): (88, 512),
          (256, 16, 128, 2): (172, 1024), (256, 32, 128, 2): (172, 1024), (256, 16, 256, 2): (344, 1024)}
TIER1_KERNEL = "k_sample<64, 1, 1024, 1368, 64, 2, 1>"
TIER2_KERNEL = "k_sample<64, 1, 6144, 8192, 64, 1, 2>"
TIER3_KERNEL = "k_sample<1024, 1, 1, 1, 8192, 2, 3>"


def tier_kernel_names(opts):
    key = (opts.get("threads_per_block", 64), opts.get("slots_per_block", 4), opts.get("visited_threshold", 192),
           opts.get("quads_per_lane", 1))
    hcap, icap = _TIER0[key]
    t0 = "k_sample<%d, %d, %d, %d, %d, %d, 0>" % (key[0], key[1], key[2], hcap, icap, key[3])
    return [t0, TIER1_KERNEL, TIER2_KERNEL, TIER3_KERNEL]


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def random_access_probe(dev, table_log2=33, reps=5):
    """Achievable random-access HBM bandwidth: the library's probe reads 2^26 rows at uniformly
    random positions of an 8 GiB table, far above the last-level caches, at the sampler's two
    random granules (8-byte row bounds, 32-byte edge quads) and at 64 and 128 bytes (half and
    whole cache lines).  Bytes counted: the rows read.  Best of `reps`, timed with events on
    torch's stream (where the probe is launched)."""
    import torch

    from paper_1709_03565_amd import skis
    table = torch.zeros(1 << table_log2, dtype=torch.uint8, device=dev)
    sink = torch.zeros(1, dtype=torch.int32, device=dev)
    reads = 1 << 26
    res = {"probe": "skis_probe_random_read: 2^26 uniformly random rows of an 8 GiB table, bytes of the rows read"}
    for rb in (8, 32, 64, 128):
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


def load_graph(name, dev):
    """Device tensors (row_ptr, col, w) and a host namespace for a workload."""
    import torch

    from paper_1709_03565_amd import inputs
    wl = inputs.WORKLOADS[name]
    if wl.get("device_graph"):
        # drawn on the GPU: a host build of this size takes minutes
        rp, col, w = inputs.chung_lu_graph_device(wl["n"], wl["m"], wl["beta"], wl["seed"], wl["model"], dev)
        torch.cuda.synchronize()
        g = types.SimpleNamespace(n=wl["n"], m=wl["m"], row_ptr=None, col=None, w=None)
    else:
        g = inputs.workload_graph(name)
        rp = torch.from_numpy(g.row_ptr).to(dev)
        col = torch.from_numpy(g.col).to(dev)
        w = torch.from_numpy(g.w).to(dev)
    return g, rp, col, w


LT_KERNELS = ["k_lt_walk", "k_lt_long"]


def tier_lines(infos, names, workload, lt=False):
    """Per sampler tier: the launch's algorithmic bytes over its HIP-event time (mean over
    the timed steps), against the HBM peak.  Linear threshold: the walk and long-walk kernels."""
    out = []
    for t in range(2 if lt else 4):
        ms = sum(getattr(x, "ms_tier%d" % t) for x in infos) / len(infos)
        inf = infos[-1]
        b = launch_bytes(inf, t, lt)
        gbs = b / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
        out.append({"tier": t, "kernel": names[t], "launch_ms": ms, "alg_bytes_per_launch": b,
                    "achieved_gbs": gbs, "frac_of_hbm_peak": gbs / HBM_PEAK_GBS,
                    "samples_finished": inf.tier_samples[t], "entries_finished": inf.tier_entries[t],
                    "edges_swept": inf.tier_swept[t], "nodes_expanded": inf.tier_items[t],
                    "traffic": measured_traffic(names[t], workload)})
        if lt:
            out[-1]["picks_drawn"] = out[-1].pop("edges_swept")
    return out


def run_steps(name, rp, col, w, T, opts, steps, warmup, set_ptr=None, set_nodes=None, k=100, build_only=False):
    import torch

    from paper_1709_03565_amd import inputs, skis

    def step():
        if build_only:
            sk = skis.build_sketch(rp, col, w, T, inputs.SAMPLE_SEED, build_inverse_index=0, **opts)
            inf = sk.info()
            sk.free()
            return inf
        sk = skis.build_sketch(rp, col, w, T, inputs.SAMPLE_SEED, **opts)
        sk.estimate(set_ptr, set_nodes)
        sk.greedy(k)
        inf = sk.info()
        sk.free()
        return inf

    for i in range(warmup):
        inf = step()
        log("%s warmup %d: %s" % (name, i, inf))
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for i in range(steps):
        infos.append(step())
        log("%s step %d done" % (name, i))
    torch.cuda.synchronize()
    return infos, time.perf_counter() - t0


def stage_means(infos):
    keys = ["ms_preprocess", "ms_roots", "ms_sample", "ms_tier0", "ms_tier1", "ms_tier2", "ms_tier3", "ms_compact",
            "ms_inverse"]
    return {k: round(sum(getattr(x, k) for x in infos) / len(infos), 3) for k in keys}


def oracle_baseline(g, rp, col, w, T, budget_s=20.0, build_only=True, sets=None, k=100, model=0):
    """The oracle (plain C, test infrastructure) on a bounded prefix of the same workload's
    sample ids, with every host thread the process may use and with one: preprocessing is
    timed once, sampling per sample, and the rate is extrapolated to the T samples of a step.
    For a whole-path step the oracle's inverse index, estimates and greedy on the prefix
    sketch are timed too and scaled by T / prefix."""
    import numpy as np

    import oracle
    threads = len(os.sched_getaffinity(0))
    if g.row_ptr is None:
        hrp, hcol, hw = rp.cpu().numpy(), col.cpu().numpy(), w.cpu().numpy()
    else:
        hrp, hcol, hw = g.row_ptr, g.col, g.w
    log("cpu baseline: oracle preprocessing (one thread)")
    t = time.perf_counter()
    prep = oracle.Prepared(hrp, hcol, hw, model=model)
    t_prep = time.perf_counter() - t
    # size the prefix for about budget_s seconds of sampling with every thread
    n0 = 1 << 13
    t = time.perf_counter()
    prep.sample(1, 0, n0, nthreads=threads)
    rate = n0 / max(time.perf_counter() - t, 1e-4)
    Ns = int(min(max(rate * budget_s, 1 << 14), 1 << 20, T))
    Ns = 1 << int(math.log2(Ns))
    log("cpu baseline: sampling ids [0, %d) with %d threads" % (Ns, threads))
    t = time.perf_counter()
    sk = prep.sample(1, 0, Ns, nthreads=threads)
    t_samp = time.perf_counter() - t
    per_sample = t_samp / Ns
    # one thread, on a smaller prefix
    N1 = max(1 << 10, min(Ns // max(threads, 1), 1 << 16))
    N1 = 1 << int(math.log2(N1))
    t = time.perf_counter()
    prep.sample(1, 0, N1, nthreads=1)
    per_sample_1 = (time.perf_counter() - t) / N1
    t_query = 0.0
    if not build_only:
        q = prep.q()
        set_ptr, set_nodes = sets
        t = time.perf_counter()
        oracle.inverse(g.n, sk.sample_ptr, sk.nodes)
        oracle.estimate(g.n, sk.sample_ptr, sk.nodes, q, sk.Gamma, set_ptr=set_ptr, set_nodes=set_nodes)
        oracle.greedy(g.n, sk.sample_ptr, sk.nodes, q, sk.Gamma, k)
        t_query = time.perf_counter() - t
    prep.close()
    t_full = t_prep + per_sample * T + t_query * (T / Ns)
    t_full_1 = t_prep + per_sample_1 * T + t_query * (T / Ns)
    log("cpu baseline: prep %.2fs, %.3g s/sample (%d threads), %.3g s/sample (1 thread) -> %.3g samples/s" %
        (t_prep, per_sample, threads, per_sample_1, T / t_full))
    return {
        "value": T / t_full,
        "unit": "samples/s",
        "cores": threads,
        "kind": "oracle",
        "cpu_model": cpu_model(),
        "sample": ("oracle (plain C, %d threads) on sample ids [0, %d) of the same workload: preprocessing "
                   "%.2f s once (one thread) + %.3g s/sample sampling%s, extrapolated to T=%d samples"
                   % (threads, Ns, t_prep, per_sample,
                      "" if build_only else ", plus its inverse index, estimates and greedy k=%d on that "
                      "sketch (%.2f s) scaled by T/%d" % (k, t_query, Ns), T)),
        "sampling_only_samples_per_s": 1.0 / per_sample,
        "single_thread": {"value": T / t_full_1, "sampling_only_samples_per_s": 1.0 / per_sample_1,
                          "sample": "sample ids [0, %d) with one thread" % N1},
    }


def serving_run(sk, n, T, name, rate, duration, warm_s=1.0):
    """Open-loop serving over a resident sketch: Poisson arrivals, Zipf(1.5) set sizes in
    1..1000, latency from scheduled arrival to the result in host memory; the first warm_s
    seconds are warm-up.  Every result is compared with skis_estimate of the same sets in
    one plain batch call (alone vs in the mix)."""
    import numpy as np
    import torch

    from paper_1709_03565_amd import inputs, skis
    nq = int(round(rate * (warm_s + duration)))
    set_ptr, set_nodes, arrival = inputs.serving_trace(n, nq, rate, seed=11)
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
    acov, aest = sk.estimate(torch.from_numpy(set_ptr).cuda(), torch.from_numpy(set_nodes).cuda())
    same = bool(np.array_equal(acov.cpu().numpy().astype(np.uint64), cov) and np.array_equal(aest.cpu().numpy(), est))
    node_ptr = sk.inverse()[0].cpu().numpy()
    degH = np.diff(node_ptr)
    work = np.add.reduceat(degH[set_nodes], set_ptr[:-1]) if len(set_nodes) else np.zeros(nq, np.int64)
    wm = work[meas]
    heavy = wm >= np.percentile(wm, 99)
    res = {
        "workload": "%s resident sketch (T=%d); open-loop Poisson %.0f q/s, Zipf(1.5) set sizes in 1..1000, "
                    "members uniform; %.0f s warm-up + %.0f s measured" % (name, T, rate, warm_s, duration),
        "p50_us": float(np.percentile(lm, 50)),
        "p90_us": float(np.percentile(lm, 90)),
        "p99_us": float(np.percentile(lm, 99)),
        "p999_us": float(np.percentile(lm, 99.9)),
        "max_us": float(lm.max()),
        "offered_qps": rate,
        "achieved_qps": float(achieved),
        "queries_measured": int(meas.sum()),
        "replay_wall_s": wall,
        "batches": st["batches"],
        "mean_batch": st["queries"] / max(st["batches"], 1),
        "max_batch": st["max_batch"],
        "batch_hist_pow2": st["batch_hist"],
        "server_device_bytes": st["device_bytes"],
        "alone_vs_mix_identical": same,
        "work_entries_p50": float(np.percentile(wm, 50)),
        "work_entries_p99": float(np.percentile(wm, 99)),
        "work_entries_max": int(wm.max()),
        "p50_us_heaviest_1pct": float(np.percentile(lm[heavy], 50)),
        "p99_us_rest": float(np.percentile(lm[~heavy], 99)),
    }
    log("serve: p50 %.1f us p99 %.1f us achieved %.0f q/s, %d batches (mean %.2f), identical alone/mix: %s" %
        (res["p50_us"], res["p99_us"], achieved, st["batches"], res["mean_batch"], same))
    return res


def ris_comparison(g, rp, col, w, T, set_ptr, set_nodes):
    """RIS (Sec. 2.3.1) beside IIS on the same graph, T samples each: the fraction of singular
    RIS samples against 1 - Gamma / n (Sec. 3.1), and per query set the variance of one
    sample's estimate, Var[Y] = n^2 p_R (1 - p_R) for RIS and Var[Z] = Gamma^2 p_I (1 - p_I)
    for IIS (Lemma lem:zvar: Var[Z] <= Var[Y]), with p the coverage fractions of the sketches."""
    import numpy as np

    from paper_1709_03565_amd import inputs, skis
    iis = skis.build_sketch(rp, col, w, T, inputs.SAMPLE_SEED)
    ris = skis.build_sketch(rp, col, w, T, inputs.SAMPLE_SEED, ris_mode=1)
    ii, ri = iis.info(), ris.info()
    sizes = np.diff(ris.export()[0].cpu().numpy())
    singular = float((sizes == 1).mean())
    ci = iis.estimate(set_ptr, set_nodes)[0].cpu().numpy().astype(np.float64) / T
    cr = ris.estimate(set_ptr, set_nodes)[0].cpu().numpy().astype(np.float64) / T
    vz = ii.Gamma ** 2 * ci * (1 - ci)
    vy = float(g.n) ** 2 * cr * (1 - cr)
    ratio = vz / np.maximum(vy, 1e-300)
    ris.free()
    # greedy identifiability (the synthetic analogue of the paper's Fig. 3): k seeds picked on
    # small IIS and RIS sketches (5 sample seeds each), each seed set judged by Eq. eq21 on the
    # large IIS sketch of the step's seed
    import torch
    k = 50
    ptr = torch.tensor([0, k], dtype=torch.int64, device="cuda")
    quality = []
    for Ts in (1000, 10000, 100000):
        got = {"iis": [], "ris": []}
        for r in range(5):
            for mode in ("iis", "ris"):
                sk = skis.build_sketch(rp, col, w, Ts, 1000 + 10 * r + (mode == "ris"), ris_mode=int(mode == "ris"))
                seeds = sk.greedy(k)[0]
                sk.free()
                got[mode].append(float(iis.estimate(ptr, seeds.to(torch.int32))[1][0]))
        quality.append({"T": Ts, "k": k, "iis_mean": float(np.mean(got["iis"])), "ris_mean": float(np.mean(got["ris"])),
                        "iis": got["iis"], "ris": got["ris"]})
        log("greedy on T=%d: I_hat(seeds) IIS %.0f, RIS %.0f (judged on the T=%d IIS sketch)" %
            (Ts, quality[-1]["iis_mean"], quality[-1]["ris_mean"], T))
    iis.free()
    res = {"T": T, "singular_fraction": singular, "one_minus_gamma_over_n": 1.0 - ii.Gamma / g.n,
           "var_ratio_z_over_y_median": float(np.median(ratio)), "var_ratio_z_over_y_max": float(ratio.max()),
           "queries_var_z_le_var_y": int((vz <= vy).sum()), "queries": int(len(ci)),
           "ris_sampler_ms": ri.ms_tier0 + ri.ms_tier1 + ri.ms_tier2 + ri.ms_tier3, "ris_entries": ri.entries,
           "iis_sampler_ms": ii.ms_tier0 + ii.ms_tier1 + ii.ms_tier2 + ii.ms_tier3, "iis_entries": ii.entries,
           "greedy_quality": quality}
    log("RIS vs IIS: singular %.4f (1 - Gamma/n %.4f), Var[Z]/Var[Y] median %.3f max %.3f" %
        (singular, res["one_minus_gamma_over_n"], res["var_ratio_z_over_y_median"], res["var_ratio_z_over_y_max"]))
    return res


def full_step_workload(name, dev, steps, warmup, k, queries, plain_compare, serve_args=None, ris_compare=False,
                       dssa_k=0):
    """A whole-path step (build with inverse index, estimates, greedy) on a host-generated
    workload, with the tier lines; optionally the plain form and a serving run."""
    import torch

    from paper_1709_03565_amd import inputs, skis
    wl = inputs.WORKLOADS[name]
    T = wl["T"]
    lt = wl["model"] == "lt"
    build_only = bool(wl.get("build_only"))
    opts = {"model": 1} if lt else {}
    t = time.perf_counter()
    g, rp, col, w = load_graph(name, dev)
    torch.cuda.empty_cache()
    log("%s graph ready in %.1fs" % (name, time.perf_counter() - t))
    sets = inputs.random_sets(g.n, queries, 50, seed=7)
    sp_np, sn_np = inputs.sets_to_csr(sets)
    set_ptr, set_nodes = torch.from_numpy(sp_np).to(dev), torch.from_numpy(sn_np).to(dev)
    infos, elapsed = run_steps(name, rp, col, w, T, opts, steps, warmup, set_ptr, set_nodes, k, build_only)
    inf = infos[-1]
    samp_ms = sum(x.ms_roots + x.ms_sample + x.ms_compact for x in infos) / len(infos)
    step_text = ("build_sketch without the inverse index" if build_only else
                 "build_sketch + inverse index + %d estimates + greedy k=%d" % (queries, k))
    res = {"workload": "%s: n=%d m=%d beta=%g %s weights, %s sampler, T=%d%s; step = %s"
                       % (name, g.n, g.m, wl["beta"], wl["model"].upper(),
                          "linear threshold (Sec. 6)" if lt else "independent cascade", T,
                          ", graph drawn on the GPU" if wl.get("device_graph") else "", step_text),
           "ms_per_step": elapsed * 1000.0 / steps, "samples_per_s": T * steps / elapsed,
           "sampling_samples_per_s": T / (samp_ms * 1e-3), "edges_probed_per_s": inf.probed_total * steps / elapsed,
           "entries": inf.entries, "probed_total": inf.probed_total, "stages_ms": stage_means(infos),
           "tiers": tier_lines(infos, LT_KERNELS if lt else tier_kernel_names({}), name, lt)}
    if plain_compare:
        sk = skis.build_sketch(rp, col, w, T, inputs.SAMPLE_SEED, form=1, build_inverse_index=0)
        pinf = sk.info()
        sk.free()
        pers = sum(x.ms_tier0 + x.ms_tier1 + x.ms_tier2 + x.ms_tier3 for x in infos) / len(infos)
        res["plain_form"] = {"sampler_ms": pinf.ms_tier0, "levels": pinf.plain_levels, "persistent_sampler_ms": pers,
                             "speedup_persistent_over_plain": pinf.ms_tier0 / pers}
        log("%s plain form: sampler %.1f ms over %d level launches; persistent %.1f ms" %
            (name, pinf.ms_tier0, pinf.plain_levels, pers))
    if ris_compare:
        res["ris_comparison"] = ris_comparison(g, rp, col, w, T, set_ptr, set_nodes)
    if dssa_k:
        # D-SSA on SKIS sketches with the paper's IM settings (eps = 0.5, delta = 1/n)
        torch.cuda.synchronize()
        t = time.perf_counter()
        seeds, dinfo, _ = skis.im_dssa(rp, col, w, dssa_k, 0.5, 1.0 / g.n, inputs.SAMPLE_SEED)
        torch.cuda.synchronize()
        res["im_dssa"] = dict(dinfo, k=dssa_k, eps=0.5, delta=1.0 / g.n, seconds=time.perf_counter() - t)
        log("%s D-SSA k=%d: %.3f s, T=%d, %d iterations, stopped %d, I_hat %.1f" %
            (name, dssa_k, res["im_dssa"]["seconds"], dinfo["T"], dinfo["iterations"], dinfo["stopped"],
             dinfo["est_check"]))
    if serve_args is not None:
        sk = skis.build_sketch(rp, col, w, T, inputs.SAMPLE_SEED)
        res["serving"] = serving_run(sk, g.n, T, name, *serve_args)
        sk.free()
    del rp, col, w
    torch.cuda.empty_cache()
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cl40m_wc")
    ap.add_argument("--samples", type=int, default=0, help="override T (default: the workload's)")
    ap.add_argument("--queries", type=int, default=100)
    ap.add_argument("--k", type=int, default=100)
    ap.add_argument("--slots", type=int, default=0)
    ap.add_argument("--visited", type=int, default=0)
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--big-row", type=int, default=0)
    ap.add_argument("--qpl", type=int, default=0, help="edge quads per lane per sweep in the first tier (1 or 2)")
    ap.add_argument("--form", type=int, default=0, help="0: persistent sampler, 1: plain, 2: captured")
    ap.add_argument("--chunk", type=int, default=0, help="captured form: sample ids per graph replay (0: the library's)")
    ap.add_argument("--autotune", action="store_true", help="autotune the first tier's shape on the workload first")
    ap.add_argument("--no-extras", action="store_true",
                    help="the headline workload only (no other workloads, serving run or random-read probe)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cache-gib", type=float, default=0.0,
                    help="the library's idle-block cache and pool limits in GiB (0: its defaults)")
    ap.add_argument("--no-captured", action="store_true",
                    help="skip the captured-form build beside the headline (profiling runs: only the timed launches)")
    ap.add_argument("--serve", action="store_true",
                    help="serving benchmark alone: open-loop Poisson query stream against a resident sketch")
    ap.add_argument("--rate", type=float, default=50000.0, help="serving: offered queries per second")
    ap.add_argument("--duration", type=float, default=0.0,
                    help="serving: measured seconds after 1 s of warm-up (default 10 with --serve, 3 as an extra)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (for scaling HBM byte counters) and exit")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py measures one GPU only: the sketch shards by sample id with no communication, "
              "and this benchmark runs and reports a single GPU (got --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1709_03565_amd import inputs, skis

    if args.calibrate_copy:
        nbytes = args.calibrate_copy << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": nbytes, "launches": 3}), flush=True)
        return

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    skis.lib()  # fails loudly if the HIP library is missing
    if args.cache_gib > 0:
        skis.set_memory_limits(int(args.cache_gib * (1 << 30)), int(args.cache_gib * (1 << 30)))

    if args.serve:
        name = "cl4m_tri" if inputs.WORKLOADS[args.workload].get("build_only") else args.workload
        T = args.samples or inputs.WORKLOADS[name]["T"]
        g, rp, col, w = load_graph(name, dev)
        sk = skis.build_sketch(rp, col, w, T, inputs.SAMPLE_SEED)
        r = serving_run(sk, g.n, T, name, args.rate, args.duration or 10.0)
        line = {"metric": "SKIS serving latency p99", "value": r["p99_us"], "unit": "us", "n_gpus": 1,
                "higher_is_better": False, "vs_baseline": None, "dtype": "u64/f64", "data": "synthetic",
                "config": {"workload": "%s: n=%d m=%d; " % (name, g.n, g.m) + r["workload"]}}
        line.update(r)
        print(json.dumps(line), flush=True)
        return

    name = args.workload
    wl = inputs.WORKLOADS[name]
    T = args.samples or wl["T"]
    build_only = bool(wl.get("build_only"))
    lt = wl["model"] == "lt"
    log("workload", name, wl, "T", T)
    t = time.perf_counter()
    g, rp, col, w = load_graph(name, dev)
    torch.cuda.empty_cache()  # the graph generator's temporaries go back to the device
    log("graph ready in %.1fs: n=%d m=%d" % (time.perf_counter() - t, g.n, g.m))
    opts = {}
    for key, val in (("slots_per_block", args.slots), ("visited_threshold", args.visited),
                     ("threads_per_block", args.threads), ("big_row", args.big_row), ("quads_per_lane", args.qpl),
                     ("form", args.form), ("chunk_samples", args.chunk)):
        if val:
            opts[key] = val
    if lt:
        opts["model"] = 1
    tuned = None
    if args.autotune and args.form == 0 and not lt:
        from paper_1709_03565_amd import autotune
        tuned = autotune.autotune(rp, col, w, pilot_samples=T, log=log)
        opts.update(autotune.options_from(tuned))
        log("autotuned options: %s (%.2f ms on the pilot)" % (autotune.options_from(tuned), tuned["ms"]))
    sets = inputs.random_sets(g.n, args.queries, 50, seed=7)
    sp_np, sn_np = inputs.sets_to_csr(sets)
    set_ptr, set_nodes = torch.from_numpy(sp_np).to(dev), torch.from_numpy(sn_np).to(dev)
    torch.cuda.synchronize()
    infos, elapsed = run_steps(name, rp, col, w, T, opts, args.steps, args.warmup, set_ptr, set_nodes, args.k,
                               build_only)
    inf = infos[-1]
    ms_step = elapsed * 1000.0 / args.steps
    value = T * args.steps / elapsed
    names = LT_KERNELS if lt else tier_kernel_names(opts)
    tiers = tier_lines(infos, names, name, lt)
    dom = max(tiers, key=lambda x: x["launch_ms"])
    samp_ms = sum(x.ms_roots + x.ms_sample + x.ms_compact for x in infos) / len(infos)
    sampler_ms = sum(x.ms_tier0 + x.ms_tier1 + x.ms_tier2 + x.ms_tier3 for x in infos) / len(infos)
    b_chain = 60 * T + 24 * inf.entries if lt else sample_bytes(T, inf.entries, inf.probed_total)
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
            "workload": "%s: directed Chung-Lu n=%d m=%d beta=%g, %s weights fp32, T=%d %s IIS samples, Philox seed %d; "
                        % (name, g.n, g.m, wl["beta"], wl["model"].upper(), T,
                           "linear threshold" if lt else "independent cascade", inputs.SAMPLE_SEED)
                        + ("graph drawn on the GPU; step = build_sketch without the inverse index" if build_only else
                           "step = build_sketch + inverse index + %d estimates (|S| 1-50) + greedy k=%d"
                           % (args.queries, args.k)),
            "T": T, "n": g.n, "m": g.m,
        },
        "edges_probed_per_s": inf.probed_total * args.steps / elapsed,
        "sampling_samples_per_s": T / (samp_ms * 1e-3),
        "sampling_note": "T over roots + sampler + compaction (preprocessing and inverse index excluded)",
        "entries": inf.entries,
        "probed_total": inf.probed_total,
        "deferred": inf.deferred,
        "deferred_global": inf.deferred_global,
        "deferred_bitmap": inf.deferred_bitmap,
        "stages_ms": stage_means(infos),
        "roofline": {
            "bound": "hbm",
            "kernel": dom["kernel"],
            "achieved": dom["achieved_gbs"],
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": dom["achieved_gbs"] / HBM_PEAK_GBS,
            "traffic": dom["traffic"],
            "alg_bytes_per_launch": dom["alg_bytes_per_launch"],
            "launch_ms": dom["launch_ms"],
            "note": ("the LT walk kernel with the longest launch; bytes = 60 per sample + 24 per node" if lt else
                     "the sampler tier with the longest launch; bytes = 40 per finished sample + 4 per staged "
                     "node + 8 per expanded node + 8 per swept in-edge of that launch"),
            "sampler_alg_bytes": b_chain,
            "sampler_ms": sampler_ms,
            "sampler_gbs": b_chain / (sampler_ms * 1e-3) / 1e9,
        },
        "tiers": tiers,
    }
    if tuned is not None:
        line["config"]["sampler_options"] = autotune.options_from(tuned)
    if args.form == 0 and not lt and not args.no_captured:
        # the captured form: the same chain captured into a HIP graph, replayed per chunk
        sk = skis.build_sketch(rp, col, w, T, inputs.SAMPLE_SEED, form=2, build_inverse_index=0, **opts)
        cinf = sk.info()
        sk.free()
        line["captured_form"] = {"sampler_ms": cinf.ms_tier0, "graph_replays": cinf.graph_replays,
                                 "chunk_samples": -(-T // cinf.graph_replays), "persistent_sampler_ms": sampler_ms}
        log("captured form: sampler %.1f ms over %d graph replays; persistent %.1f ms" %
            (cinf.ms_tier0, cinf.graph_replays, sampler_ms))
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = oracle_baseline(g, rp, col, w, T, build_only=build_only,
                                               sets=(sp_np, sn_np), k=args.k, model=1 if lt else 0)
    del rp, col, w
    torch.cuda.empty_cache()
    if not args.no_extras:
        extras = {}
        for other in ("cl1m_wc", "cl4m_tri", "cl40m_lt"):
            if other == name:
                continue
            serve_args = (args.rate, args.duration or 3.0) if other == "cl4m_tri" else None
            extras[other] = full_step_workload(other, dev, args.steps, args.warmup, args.k, args.queries,
                                               plain_compare=(other == "cl1m_wc"), serve_args=serve_args,
                                               ris_compare=(other == "cl1m_wc"),
                                               dssa_k=100 if other == "cl4m_tri" else 0)
        line["workloads"] = extras
        if "cl4m_tri" in extras:
            line["serving"] = extras["cl4m_tri"].pop("serving")
        try:
            ra = random_access_probe(dev)
            ra["dominant_frac_of_32B"] = dom["achieved_gbs"] / ra["rows_32B_gbs"]
            ra["dominant_frac_of_128B"] = dom["achieved_gbs"] / ra["rows_128B_gbs"]
            log("random-access probe: %.0f / %.0f / %.0f / %.0f GB/s in 8/32/64/128-B rows" %
                (ra["rows_8B_gbs"], ra["rows_32B_gbs"], ra["rows_64B_gbs"], ra["rows_128B_gbs"]))
        except Exception as ex:  # a measurement aid: its failure does not void the step's numbers
            ra = {"error": str(ex).splitlines()[0]}
            log("random-access probe failed:", ra["error"])
        line["random_access"] = ra
    print(json.dumps(line), flush=True)
    release_device_memory()


def release_device_memory():
    """Hands the library's idle blocks and pool and torch's cached blocks back to the driver
    before the process ends: a process started right after one that exits holding them (about
    130 GB at 1.4B edges) met memory the driver was still reclaiming and took 150 ms more a
    step."""
    import torch

    from paper_1709_03565_amd import skis
    torch.cuda.synchronize()
    skis.release_cached_memory()
    torch.cuda.empty_cache()
    torch.cuda.synchronize()


if __name__ == "__main__":
    main()
