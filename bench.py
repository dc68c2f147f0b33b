"""Benchmark: edges/s of the full 15-orbit non-induced count on one MI355X.

One step = one niorca_count call on a device-resident CSR (degree orientation,
Stage I, Stage II, Stage III and the equations); inputs are in HBM before the
timed region starts, outputs stay there.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload chung_lu_4m]
                    [--forms all|none] [--cpu-budget S]

Prints one JSON line.  `value` is the plain form on the workload; `forms` adds
the degree-binned and MLP-binned forms (on the workload and on R-MAT scale 22)
and the batched form (50,000 small graphs, hipGraph-captured, with the tuned
knobs of paper_2606_29651_amd/tuning.txt; --retune searches them again), next to
the plain form on the same graphs counted as one disjoint union.
`roofline` is for the dominant kernel of the timed steps: its algorithmic bytes
(the CSR words and row metadata the method itself must read for the work units
that launch processed, reported by the library's work classes) over its HIP-event
duration on the launching stream, against 8 TB/s and against the copy bandwidth
measured in the same run.  `cpu_baseline` times the CPU oracle's three stages:
Stage I over the whole graph, Stages II and III on a bounded random vertex sample
scaled to all vertices; it also holds the complete three-stage run on the tiny
Erdos-Renyi configuration on all cores and on one.
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

HBM_PEAK_GBS = 8000.0
TUNE_FILE = os.path.join(ROOT, "paper_2606_29651_amd", "tuning.txt")
# The paper's own figure for its method (multicore CPU; no absolute rates are printed).
PAPER_CONTEXT = ("NI-ORCA reports up to 30x over sequential orbit counters (EVOKE, ORCA, JESSE, CORA) at 32-64 "
                 "threads on 2x AMD EPYC 7713 (128 cores) and 2x Intel Xeon Gold 6438Y+ (64 cores), eight "
                 "real-world graphs of 12.5k-16.5M edges; not comparable with this machine or these graphs")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# Algorithmic bytes per unit, per kernel:
#   Stage I/II probe kernels: 4 B per probe (one N+(v) entry), 12 B per N+(u) entry
#     (the entry and the two row offsets of v);
#   4-cycle kernels: 4 B per wedge (the key, one N+(v) entry) and 16 B per row slot
#     (neighbour id, segment bounds, the middle's credit).
KERNEL_CLASS = {"probe_thread": "tri_thread", "probe_wave": "tri_wave", "probe_block": "tri_block",
                "probe_large": "tri_large", "ql_wave": "ql_wave", "ql_block": "ql_block",
                "ql_global": "ql_global", "qh_wave": "qh_wave", "qh_block": "qh_block",
                "qh_dense": "qh_dense", "qh_global": "qh_global", "probe_group": "tri_group"}


# kernel names of the bench's per-kernel timings -> device symbol prefixes under rocprofv3
PROF_NAME = {"probe_thread": "k_probe_thread<0>", "probe_wave": "k_probe_wave<0>", "probe_block": "k_probe_block<0>",
             "probe_large": "k_probe_large<0,", "ql_wave": "k_q_wave<0>", "ql_block": "k_q_block<0>",
             "ql_global": "k_q_global<0>", "qh_wave": "k_qh_wave", "qh_block": "k_qh_block",
             "qh_dense": "k_q_dense", "qh_global": "k_q_global<1>", "probe_group": "k_probe_group<0>"}
CSRC = os.path.join(ROOT, "paper_2606_29651_amd", "csrc")


def source_digest():
    """sha256 over the kernel sources: byte counters taken on other sources are stale."""
    import hashlib
    h = hashlib.sha256()
    for f in sorted(os.listdir(CSRC)):
        if f.endswith((".hip", ".hpp")):
            with open(os.path.join(CSRC, f), "rb") as fh:
                h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def _pmc_per_kernel(path):
    """Counter sum and dispatch count per device symbol from a rocprofv3 counter CSV."""
    import csv
    tot, calls = {}, {}
    with open(path) as fh:
        for r in csv.DictReader(fh):
            name = r["Kernel_Name"].replace("void ", "", 1)
            tot[name] = tot.get(name, 0.0) + float(r["Counter_Value"])
            calls.setdefault(name, set()).add(r["Dispatch_Id"])
    return {k: (tot[k], len(calls[k])) for k in tot}


def traffic_summary(fetch_csv, write_csv, copy_fetch_csv, copy_write_csv, copy_mib):
    """Text summary of HBM bytes per launch for each timed kernel, the counters scaled
    by what they read for a copy of known size (copy_mib MiB read and written)."""
    f, w = _pmc_per_kernel(fetch_csv), _pmc_per_kernel(write_csv)
    cf, cw = _pmc_per_kernel(copy_fetch_csv), _pmc_per_kernel(copy_write_csv)
    pick = lambda d: next(v for k, v in d.items() if "direct_copy_kernel" in k)
    known_kib = copy_mib * 1024.0
    (cfs, cfn), (cws, cwn) = pick(cf), pick(cw)
    fscale, wscale = known_kib / (cfs / cfn), known_kib / (cws / cwn)
    lines = [f"source_digest {source_digest()}", f"fetch_scale {fscale:.4f}", f"write_scale {wscale:.4f}"]
    for short, sym in PROF_NAME.items():
        fk = [v for k, v in f.items() if k.startswith(sym)]
        wk = [v for k, v in w.items() if k.startswith(sym)]
        if not fk or not wk:
            continue
        fb = fscale * 1024.0 * sum(x[0] for x in fk) / sum(x[1] for x in fk)
        wb = wscale * 1024.0 * sum(x[0] for x in wk) / sum(x[1] for x in wk)
        lines.append(f"kernel {short} fetch_bytes {fb:.0f} write_bytes {wb:.0f}")
    return "\n".join(lines)


SQ_COLS = ["SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_LDS", "SQ_INSTS_VMEM_RD",
           "SQ_INSTS_VMEM_WR", "SQ_LDS_BANK_CONFLICT", "SQ_WAIT_ANY", "SQ_WAVE_CYCLES"]


def counter_summary(paths):
    """Text table of shader-sequencer counters per dispatch for each timed kernel, from
    rocprofv3 --pmc counter CSVs (counters summed over the chip), with two ratios:
    SALU per VALU instruction and the fraction of wave cycles spent waiting."""
    import csv
    acc, calls = {}, {}
    for path in paths:
        with open(path) as fh:
            for r in csv.DictReader(fh):
                name = r["Kernel_Name"].replace("void ", "", 1)
                short = next((k for k, sym in PROF_NAME.items() if name.startswith(sym)), None)
                if short is None:
                    continue
                key = (short, r["Counter_Name"])
                acc[key] = acc.get(key, 0.0) + float(r["Counter_Value"])
                calls.setdefault(key, set()).add(r["Dispatch_Id"])
    per = {k: v / len(calls[k]) for k, v in acc.items()}
    head = ["kernel"] + [c.replace("SQ_", "").lower() for c in SQ_COLS] + ["salu/valu", "wait_frac"]
    lines = ["  ".join(f"{h:>14}" for h in head)]
    for short in PROF_NAME:
        row = [per.get((short, c)) for c in SQ_COLS]
        if row[0] is None:
            continue
        valu, salu = per.get((short, "SQ_INSTS_VALU")), per.get((short, "SQ_INSTS_SALU"))
        wait, cyc = per.get((short, "SQ_WAIT_ANY")), per.get((short, "SQ_WAVE_CYCLES"))
        ratio = f"{salu / valu:.2f}" if valu and salu is not None else "-"
        frac = f"{wait / cyc:.2f}" if cyc and wait is not None else "-"
        lines.append("  ".join([f"{short:>14}"] + [f"{v:14.4g}" if v is not None else f"{'-':>14}" for v in row]
                               + [f"{ratio:>14}", f"{frac:>14}"]))
    return "\n".join(lines)


def kernel_summary(path, top=24):
    """Text table of a rocprofv3 --kernel-trace --stats run_kernel_stats.csv: calls,
    average and total duration and share of each kernel, the top ones by total time."""
    import csv
    rows = []
    with open(path) as fh:
        for r in csv.DictReader(fh):
            name = r["Name"].replace("void ", "", 1)
            name = name.split("(")[0] if "(" in name else name
            rows.append((name, int(r["Calls"]), float(r["AverageNs"]) / 1000.0, float(r["TotalDurationNs"]) / 1e6,
                         float(r["Percentage"])))
    rows.sort(key=lambda x: -x[3])
    lines = [f"{'kernel':<58}{'calls':>7}{'avg_us':>11}{'total_ms':>11}{'pct':>7}"]
    for name, calls, avg, tot, pct in rows[:top]:
        lines.append(f"{name[:57]:<58}{calls:>7}{avg:>11.1f}{tot:>11.3f}{pct:>7.2f}")
    return "\n".join(lines)


def traffic_for(workload, kernel):
    """HBM bytes per launch of kernel from profiles/traffic_<workload>.txt, or None when
    there is no such summary or the kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.txt")
    if not os.path.exists(path):
        return None
    digest, rows = None, {}
    with open(path) as fh:
        for line in fh:
            p = line.split()
            if not p or p[0].startswith("#"):
                continue
            if p[0] == "source_digest":
                digest = p[1]
            elif p[0] == "kernel":
                rows[p[1]] = int(p[3]) + int(p[5])
    if digest != source_digest():
        return None
    return rows.get(kernel)


def git_rev():
    """HEAD of the checkout bench.py runs from, or None where there is no .git."""
    import subprocess
    try:
        r = subprocess.run(["git", "rev-parse", "HEAD"], cwd=ROOT, capture_output=True, text=True, timeout=10)
        return r.stdout.strip() or None if r.returncode == 0 else None
    except (OSError, subprocess.SubprocessError):
        return None


def kernel_bytes(kernel, stats):
    cnt, work, slots = stats[KERNEL_CLASS[kernel]]
    if kernel.startswith("probe"):
        return 4 * work + 12 * slots
    return 4 * work + 16 * slots


def time_count(ni, ctx, rp, cl, out, flags, steps, warmup, timing_steps=3):
    """Milliseconds per count over `steps` counts as a caller runs them (no event
    between stages), then stage and kernel times from `timing_steps` further counts
    with per-stage and per-kernel events."""
    import torch
    for _ in range(warmup):
        ni.count(rp, cl, out=out, ctx=ctx, flags=flags)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ni.count(rp, cl, out=out, ctx=ctx, flags=flags)
    torch.cuda.synchronize()
    ms = 1000.0 * (time.perf_counter() - t0) / steps
    stages, kernels = [], []
    for _ in range(max(1, min(steps, timing_steps))):
        ni.count(rp, cl, out=out, ctx=ctx, flags=flags | ni.TIMING)
        stages.append(ctx.stage_times())
        kernels.append(ctx.kernel_times())
    torch.cuda.synchronize()
    avg_s = {k: float(np.mean([s[k] for s in stages])) for k in stages[0]}
    avg_k = {k: float(np.mean([s[k] for s in kernels])) for k in kernels[0]}
    return ms, avg_s, avg_k


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(g, budget_s: float = 15.0, seed: int = 7, seed_tiny: int = 42):
    """The CPU oracle's three stages on the same graph: Stage I (oracle.stage1) over
    every edge, then Stages II and III (oracle.stage23_at) on uniformly drawn vertices
    until about budget_s seconds have passed, scaled by n / sample.  Also the full
    three-stage oracle.count on the tiny Erdos-Renyi configuration, all threads and one."""
    import oracle
    import graphgen as gg
    oracle.build(force=False)
    threads = oracle.num_threads()
    t0 = time.perf_counter()
    tri = oracle.stage1(g.row_ptr, g.col)
    s1 = time.perf_counter() - t0
    rng = np.random.default_rng(seed)
    order = rng.permutation(g.n).astype(np.int32)
    done, s23, batch = 0, 0.0, 64
    while s23 < budget_s and done < g.n:
        xs = order[done: done + batch]
        t0 = time.perf_counter()
        oracle.stage23_at(g.row_ptr, g.col, tri, xs)
        s23 += time.perf_counter() - t0
        done += len(xs)
        batch = min(batch * 2, 1 << 16)
    del tri
    full_s = s1 + s23 * g.n / max(done, 1)
    tiny = gg.config_graph("er_tiny", seed=seed_tiny)
    tiny_rate = {}
    for t in (threads, 1):
        oracle.set_threads(t)
        best = None
        for _ in range(3):
            t0 = time.perf_counter()
            oracle.count(tiny.row_ptr, tiny.col)
            dt = time.perf_counter() - t0
            best = dt if best is None else min(best, dt)
        tiny_rate[f"threads_{t}"] = tiny.m / best
    oracle.set_threads(threads)
    return {"value": g.m / full_s, "unit": "edges/s", "cores": threads, "kind": "oracle",
            "sample": f"Stage I (sorted merges) over all {g.m} edges in {s1:.1f} s; Stages II and III on {done} "
                      f"uniformly drawn vertices in {s23:.1f} s, scaled by n/{done}",
            "cpu_model": cpu_model(),
            "er_tiny_full_edges_per_s": {k: round(v, 1) for k, v in tiny_rate.items()},
            "paper": PAPER_CONTEXT}


def stage1_work(c):
    return c[:, 0] + 4 * c[:, 1] + c[:, 2]


def base_repeats(ni, ctx, rp, cl, out, k=5):
    """ms of k single plain counts: the run-to-run spread the forms are compared against."""
    import torch
    res = []
    for _ in range(k):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ni.count(rp, cl, out=out, ctx=ctx)
        torch.cuda.synchronize()
        res.append(1000.0 * (time.perf_counter() - t0))
    return res


def judge_binning(ni, ctx, g, rp, cl, model):
    """Measured work of the Stage I/II items (shader-clock cycles per item, the
    counters' last column) under the plain, degree-binned and MLP-binned forms on a
    graph the model was not trained on: the model's error against log2(1 + cycles)
    of the plain form, and per form the spread of the item cycles (p99 and maximum
    over the mean: the load imbalance the binning is meant to reduce) and the total."""
    import torch
    out = {}
    for name, flags in (("plain", 0), ("degree", ni.BIN_DEGREE), ("mlp", ni.BIN_MLP)):
        ni.count(rp, cl, ctx=ctx, flags=flags | ni.COUNTERS)
        c = ni.work_counters(g.n, ctx=ctx)
        cyc = c[:, 6]
        keep = cyc > 0
        cy = cyc[keep].double()
        mean = float(cy.mean())
        rec = {"items": int(keep.sum()), "cycles_total": float(cy.sum()), "cycles_mean": mean,
               "p99_over_mean": float(torch.quantile(cy[torch.randperm(cy.numel(), device=cy.device)[:1 << 20]],
                                                     0.99)) / mean,
               "max_over_mean": float(cy.max()) / mean}
        if name == "plain":
            X = ni.last_features(g.n, ctx=ctx)[keep].contiguous()
            pred = ni.mlp_predict(model, X, ctx=ctx).double()
            y = torch.log2(1.0 + cy)
            err = pred - y
            rec["model_mse_log2_cycles"] = float((err * err).mean())
            rec["target_var_log2_cycles"] = float(torch.var(y))
            rec["model_r2"] = 1.0 - rec["model_mse_log2_cycles"] / rec["target_var_log2_cycles"]
            del X, pred, y, err
        out[name] = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in rec.items()}
        del c, cyc, cy
    torch.cuda.empty_cache()
    return out


def train_work_model(ni, ctx, graphs):
    """Counters of the plain form on the training graphs -> model of the measured work
    of each Stage I/II item: log2(1 + its shader-clock cycles)."""
    import torch
    Xs, ys = [], []
    for g in graphs:
        rp, cl = torch.from_numpy(g.row_ptr).cuda(), torch.from_numpy(g.col).cuda()
        ni.count(rp, cl, ctx=ctx, flags=ni.COUNTERS)
        c = ni.work_counters(g.n, ctx=ctx)
        X = ni.last_features(g.n, ctx=ctx)
        keep = c[:, 6] > 0
        Xs.append(X[keep])
        ys.append(torch.log2(1.0 + c[keep, 6].double()).float())
        del rp, cl
    X = torch.cat(Xs).contiguous()
    y = torch.cat(ys).contiguous()
    model, mse = ni.mlp_train(X, y, epochs=3, batch=8192, lr=3e-3, seed=1, ctx=ctx)
    var = float(torch.var(y.double()))
    return model, {"rows": int(X.shape[0]), "mse": mse, "target_var": var}


ER_DEFAULT = ["er_4m_8", "er_4m_16", "er_4m_32"]
ER_FULL = [f"er_{n}m_{d}" for n in (1, 2, 4, 8, 16) for d in (8, 16, 32)]


def roofline_of(kernel_ms, stats):
    dom = max(kernel_ms, key=kernel_ms.get)
    b = kernel_bytes(dom, stats)
    ach = b / (kernel_ms[dom] * 1e-3) / 1e9 if kernel_ms[dom] > 0 else 0.0
    return dom, b, ach


def er_series(args, ni, names):
    """Plain form on the Erdos-Renyi scaling series: edges/s and the dominant
    kernel's algorithmic GB/s per point."""
    import torch
    import graphgen as gg
    res = {}
    ctx = ni.Context(0)
    for name in names:
        t0 = time.time()
        g = gg.config_graph(name, seed=args.seed)
        gen_s = time.time() - t0
        rp, cl = torch.from_numpy(g.row_ptr).cuda(), torch.from_numpy(g.col).cuda()
        out = torch.empty((g.n, 15), dtype=torch.int64, device="cuda")
        ms, st, km = time_count(ni, ctx, rp, cl, out, 0, 3, 1)
        dom, b, ach = roofline_of(km, ctx.class_stats())
        res[name] = {"n": g.n, "m": g.m, "ms": round(ms, 3), "value": g.m / (ms * 1e-3),
                     "stage_ms": {k: round(v, 3) for k, v in st.items()},
                     "dominant": dom, "dominant_ms": round(km[dom], 3), "dominant_GBps": round(ach, 1)}
        log(f"[bench] {name} m={g.m} gen {gen_s:.1f}s: {ms:.2f} ms/count, {g.m / (ms * 1e-3):.3e} edges/s, "
            f"{dom} {ach:.0f} GB/s")
        del rp, cl, out
        torch.cuda.empty_cache()
    ctx.close()
    return res


def forms(args, ni, ctx, g, rp, cl, out, base_ms):
    import torch
    import graphgen as gg
    from paper_2606_29651_amd import autotune
    res = {}
    t0 = time.time()
    er = gg.config_graph("er_tiny", seed=args.seed)
    model, fit = train_work_model(ni, ctx, [er, g])
    log(f"[bench] work model trained on {fit['rows']} items, mse {fit['mse']:.3f} (target var "
        f"{fit['target_var']:.3f}) in {time.time() - t0:.1f}s")
    # thresholds of the learned binning: a small search on the training graph
    ref = out.clone()
    best = None
    # thresholds on predicted log2 item cycles (a Chung-Lu item averages about 2^17)
    for thr_t in (-99.0, 12.0):
        for thr_g in (-99.0, 12.0, 13.0, 14.0, 15.0, 16.0):
            for thr_b in (22.0, 99.0):
                ni.set_cost_model(model, thr_t, thr_b, thr_g, ctx=ctx)
                ms, _, _ = time_count(ni, ctx, rp, cl, out, ni.BIN_MLP, 2, 1)
                if best is None or ms < best[0]:
                    best = (ms, thr_t, thr_b, thr_g)
    ni.set_cost_model(model, best[1], best[2], best[3], ctx=ctx)
    res["work_model"] = {"train_rows": fit["rows"], "mse": round(fit["mse"], 4),
                         "target_var": round(fit["target_var"], 4), "thr_thread": best[1], "thr_group": best[3],
                         "thr_block": best[2]}
    deg_ms, _, _ = time_count(ni, ctx, rp, cl, out, ni.BIN_DEGREE, 3, 1)
    same_deg = bool(torch.equal(out, ref))
    mlp_ms, _, _ = time_count(ni, ctx, rp, cl, out, ni.BIN_MLP, 3, 1)
    same_mlp = bool(torch.equal(out, ref))
    res[args.workload] = {"plain": g.m / (base_ms * 1e-3), "degree": g.m / (deg_ms * 1e-3),
                          "mlp": g.m / (mlp_ms * 1e-3), "identical": same_deg and same_mlp,
                          "plain_ms_repeats": [round(x, 3) for x in base_repeats(ni, ctx, rp, cl, out)]}
    del ref
    # R-MAT scale 22: plain vs degree-binned vs MLP-binned
    t0 = time.time()
    r = gg.config_graph("rmat22", seed=args.seed)
    log(f"[bench] rmat22 n={r.n} m={r.m} generated in {time.time() - t0:.1f}s")
    rrp, rcl = torch.from_numpy(r.row_ptr).cuda(), torch.from_numpy(r.col).cuda()
    rout = torch.empty((r.n, 15), dtype=torch.int64, device="cuda")
    pl_ms, pl_st, _ = time_count(ni, ctx, rrp, rcl, rout, 0, 3, 1)
    rref = rout.clone()
    dg_ms, _, _ = time_count(ni, ctx, rrp, rcl, rout, ni.BIN_DEGREE, 3, 1)
    same = bool(torch.equal(rout, rref))
    ml_ms, _, _ = time_count(ni, ctx, rrp, rcl, rout, ni.BIN_MLP, 3, 1)
    same = same and bool(torch.equal(rout, rref))
    res["rmat22"] = {"n": r.n, "m": r.m, "plain": r.m / (pl_ms * 1e-3), "degree": r.m / (dg_ms * 1e-3),
                     "mlp": r.m / (ml_ms * 1e-3), "identical": same,
                     "plain_stage_ms": {k: round(v, 3) for k, v in pl_st.items()},
                     "plain_ms_repeats": [round(x, 3) for x in base_repeats(ni, ctx, rrp, rcl, rout)],
                     "measured_work": judge_binning(ni, ctx, r, rrp, rcl, model)}
    del rrp, rcl, rout, rref
    torch.cuda.empty_cache()
    # batched: 50,000 small graphs, tuned knobs, captured hipGraph
    t0 = time.time()
    graphs = gg.batch_mix(args.batch_graphs, 20, 2000, seed=args.seed)
    vtx_off, brp, bcol = gg.pack_batch(graphs)
    bm = int(brp[-1] // 2)
    log(f"[bench] batch of {len(graphs)} graphs, n={vtx_off[-1]} m={bm} in {time.time() - t0:.1f}s")
    tctx = ni.Context(0)
    if args.retune or not autotune.load(TUNE_FILE, "batch_mix"):
        # tune on a seeded random tenth of the batch
        pick = np.sort(np.random.default_rng(args.seed + 1).choice(len(graphs), max(1, len(graphs) // 10),
                                                                    replace=False))
        s_off, s_rp, s_col = gg.pack_batch([graphs[i] for i in pick])
        d_srp, d_scol = torch.from_numpy(s_rp).cuda(), torch.from_numpy(s_col).cuda()
        s_out = torch.empty((int(s_off[-1]), 15), dtype=torch.int64, device="cuda")
        cands = autotune.grid(bin_mode=[0, 1], heavy_k=[0, 4096, 32768], tri_wave=[32, 64],
                              qh_wave=[256, 512, 1024], ql_wave=[256, 512])
        tuned = autotune.tune(tctx, lambda: ni.count_batched(s_off, d_srp, d_scol, out=s_out, ctx=tctx), cands,
                              repeats=3)
        autotune.save(TUNE_FILE, "batch_mix", tuned["best"],
                      note=f"fastest of {len(cands)} on a random tenth of the batch, {tuned['ms']:.2f} ms")
        del d_srp, d_scol, s_out
    tctx.load_tuning(TUNE_FILE, "batch_mix")
    knobs = autotune.load(TUNE_FILE, "batch_mix")
    d_brp, d_bcol = torch.from_numpy(brp).cuda(), torch.from_numpy(bcol).cuda()
    b_out = torch.empty((int(vtx_off[-1]), 15), dtype=torch.int64, device="cuda")
    stream = torch.cuda.Stream()
    ni.count_batched(vtx_off, d_brp, d_bcol, out=b_out, ctx=tctx, stream=stream, flags=ni.GRAPH_CAPTURE)
    stream.synchronize()
    reps = 5
    t1 = time.perf_counter()
    for _ in range(reps):
        ni.count_batched(vtx_off, d_brp, d_bcol, out=b_out, ctx=tctx, stream=stream, flags=ni.GRAPH_CAPTURE)
    stream.synchronize()
    b_ms = 1000.0 * (time.perf_counter() - t1) / reps
    b_ref = b_out.clone()
    # the same launch sequence uncaptured
    t1 = time.perf_counter()
    ni.count_batched(vtx_off, d_brp, d_bcol, out=b_out, ctx=tctx, stream=stream)
    stream.synchronize()
    nb_ms = 1000.0 * (time.perf_counter() - t1)
    same = bool(torch.equal(b_out, b_ref))
    # the learned binning in place of the degree thresholds (model and thresholds of
    # the Chung-Lu search above), captured the same way
    ni.set_cost_model(model, best[1], best[2], best[3], ctx=tctx)
    tctx.set_param("bin_mode", 2)
    ni.count_batched(vtx_off, d_brp, d_bcol, out=b_out, ctx=tctx, stream=stream, flags=ni.GRAPH_CAPTURE)
    stream.synchronize()
    t1 = time.perf_counter()
    for _ in range(reps):
        ni.count_batched(vtx_off, d_brp, d_bcol, out=b_out, ctx=tctx, stream=stream, flags=ni.GRAPH_CAPTURE)
    stream.synchronize()
    bm_ms = 1000.0 * (time.perf_counter() - t1) / reps
    same = same and bool(torch.equal(b_out, b_ref))
    # and with no binning at all
    tctx.set_param("bin_mode", 0)
    ni.count_batched(vtx_off, d_brp, d_bcol, out=b_out, ctx=tctx, stream=stream, flags=ni.GRAPH_CAPTURE)
    stream.synchronize()
    t1 = time.perf_counter()
    for _ in range(reps):
        ni.count_batched(vtx_off, d_brp, d_bcol, out=b_out, ctx=tctx, stream=stream, flags=ni.GRAPH_CAPTURE)
    stream.synchronize()
    b0_ms = 1000.0 * (time.perf_counter() - t1) / reps
    same = same and bool(torch.equal(b_out, b_ref))
    tctx.close()
    # the plain form on the same graphs: niorca_count of their disjoint union (global ids)
    u_col = torch.from_numpy(bcol).cuda()
    u_col += torch.repeat_interleave(torch.from_numpy(vtx_off[:-1]).cuda().to(torch.int32),
                                     torch.from_numpy(np.diff(brp[vtx_off])).cuda())
    pctx = ni.Context(0)
    p_ms, _, _ = time_count(ni, pctx, d_brp, u_col, b_out, 0, reps, 1)
    same = same and bool(torch.equal(b_out, b_ref))
    # the plain form graph by graph (one niorca_count per graph, as a caller without
    # the batched entry would run it) on a seeded random subset, scaled to edges/s
    pick = np.sort(np.random.default_rng(args.seed + 2).choice(len(graphs), 2000, replace=False))
    sub = [graphs[i] for i in pick]
    dev = [(torch.from_numpy(x.row_ptr).cuda(), torch.from_numpy(x.col).cuda(),
            torch.empty((x.n, 15), dtype=torch.int64, device="cuda")) for x in sub]
    for (a, b, o) in dev[:20]:
        ni.count(a, b, out=o, ctx=pctx)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for (a, b, o) in dev:
        ni.count(a, b, out=o, ctx=pctx)
    torch.cuda.synchronize()
    pg_s = time.perf_counter() - t1
    pg_m = sum(x.m for x in sub)
    pctx.close()
    del dev
    res["batch_mix"] = {"graphs": len(graphs), "n": int(vtx_off[-1]), "m": bm, "captured_ms": b_ms,
                        "value": bm / (b_ms * 1e-3), "uncaptured_ms": nb_ms, "plain_union_ms": p_ms,
                        "plain_union_value": bm / (p_ms * 1e-3),
                        "plain_per_graph_value": pg_m / pg_s,
                        "mlp_binned_captured_ms": bm_ms, "mlp_binned_value": bm / (bm_ms * 1e-3),
                        "unbinned_captured_ms": b0_ms, "unbinned_value": bm / (b0_ms * 1e-3),
                        "plain_per_graph_sample": f"{len(sub)} seeded random graphs of the batch, {pg_m} edges, "
                                                  f"one niorca_count each, in {pg_s * 1000:.1f} ms",
                        "identical": same, "tuned": knobs}
    del d_brp, d_bcol, b_out, b_ref, u_col
    torch.cuda.empty_cache()
    return res


def copy_bandwidth(mib=1024, reps=10, convert=True):
    """GB/s of a plain device copy (4 B read and 4 B written per element), timed with
    events on torch's stream: an int32 -> float32 conversion kernel (convert) or a
    same-type device-to-device copy."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.arange(n, dtype=torch.int32, device="cuda")
    dst = torch.empty(n, dtype=torch.float32 if convert else torch.int32, device="cuda")
    dst.copy_(src)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        dst.copy_(src)
    b.record()
    b.synchronize()
    ms = a.elapsed_time(b) / reps
    del src, dst
    return {"elements": n, "read_bytes": 4 * n, "write_bytes": 4 * n, "ms": ms, "GBps": 8 * n / (ms * 1e-3) / 1e9}


def copy_calibration(mib):
    """A copy kernel of known traffic: 4 B read and 4 B written per element."""
    print(json.dumps({"copy_calibration": copy_bandwidth(mib, 5)}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="chung_lu_4m")
    ap.add_argument("--seed", type=int, default=42)
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--forms", default="all", choices=["all", "none"])
    ap.add_argument("--batch-graphs", type=int, default=50000)
    ap.add_argument("--retune", action="store_true",
                    help="search the batched form's knobs again and rewrite paper_2606_29651_amd/tuning.txt")
    ap.add_argument("--er-series", default="default", choices=["default", "full", "none"],
                    help="Erdos-Renyi points timed with the forms: n = 4M at average degree 8, 16, 32 "
                         "(default), all of n in {1,2,4,8,16}M x degree {8,16,32} (full), or none")
    ap.add_argument("--traffic-summary", nargs=4, metavar=("FETCH_CSV", "WRITE_CSV", "COPY_FETCH_CSV",
                                                            "COPY_WRITE_CSV"),
                    help="print the per-kernel HBM traffic summary from rocprofv3 --pmc counter CSVs of the "
                         "bench (FETCH_SIZE, WRITE_SIZE) and of --copy-calibration 1024, then exit")
    ap.add_argument("--kernel-summary", metavar="CSV",
                    help="print the per-kernel duration table of a rocprofv3 --kernel-trace --stats "
                         "run_kernel_stats.csv, then exit")
    ap.add_argument("--counter-summary", nargs="+", metavar="CSV",
                    help="print shader-sequencer counters per dispatch of each timed kernel from rocprofv3 "
                         "--pmc counter CSVs of the bench, then exit")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain int32->float32 copy of MIB MiB five times (reads and writes "
                         "MIB MiB each), to scale HBM byte counters taken under rocprofv3 --pmc")
    args = ap.parse_args()
    if args.traffic_summary:
        print(traffic_summary(*args.traffic_summary, copy_mib=1024))
        return
    if args.counter_summary:
        print(counter_summary(args.counter_summary))
        return
    if args.kernel_summary:
        print(kernel_summary(args.kernel_summary))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU path is not built",
              file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    import graphgen as gg
    import paper_2606_29651_amd as ni

    t0 = time.time()
    g = gg.config_graph(args.workload, seed=args.seed)
    log(f"[bench] generated {g.name} n={g.n} m={g.m} in {time.time() - t0:.1f}s")
    dev = torch.device("cuda:0")
    rp = torch.from_numpy(g.row_ptr).to(dev)
    cl = torch.from_numpy(g.col).to(dev)
    out = torch.empty((g.n, 15), dtype=torch.int64, device=dev)
    ctx = ni.Context(0)
    ms, stage_ms, kernel_ms = time_count(ni, ctx, rp, cl, out, 0, args.steps, args.warmup)
    stats = ctx.class_stats()
    log("[bench] stage ms " + json.dumps({k: round(v, 3) for k, v in stage_ms.items()}))
    log("[bench] kernel ms " + json.dumps({k: round(v, 3) for k, v in kernel_ms.items()}))
    dom, bytes_dom, ach = roofline_of(kernel_ms, stats)
    cb = max((copy_bandwidth(convert=c) for c in (True, False)), key=lambda r: r["GBps"])
    log(f"[bench] copy bandwidth {cb['GBps']:.0f} GB/s")
    roof = {"bound": "hbm", "kernel": dom, "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic_for(args.workload, dom),
            "copy_GBps": round(cb["GBps"], 1), "frac_of_copy": round(ach / cb["GBps"], 4),
            "kernel_ms": round(kernel_ms[dom], 4), "algorithmic_bytes": int(bytes_dom),
            "units": {"class": KERNEL_CLASS[dom], "items": stats[KERNEL_CLASS[dom]][0],
                      "work": stats[KERNEL_CLASS[dom]][1], "slots": stats[KERNEL_CLASS[dom]][2]}}
    rec = {
        "metric": "edges/sec for full 15-orbit non-induced count",
        "value": g.m / (ms * 1e-3),
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": g.n, "m": g.m, "form": "plain", "seed": args.seed,
                   "csr_sha256": g.sha256(), "source_digest": source_digest(), "git_rev": git_rev()},
        "stage_ms": {k: round(v, 4) for k, v in stage_ms.items()},
        "kernel_ms": {k: round(v, 4) for k, v in kernel_ms.items()},
        "roofline": roof,
    }
    if args.forms == "all":
        rec["forms"] = forms(args, ni, ctx, g, rp, cl, out, ms)
        if args.er_series != "none":
            rec["forms"]["er_series"] = er_series(args, ni, ER_FULL if args.er_series == "full" else ER_DEFAULT)
    rec["cpu_baseline"] = None if args.no_cpu_baseline else cpu_baseline(g, args.cpu_budget)
    print(json.dumps(rec))
    ctx.close()


if __name__ == "__main__":
    main()
