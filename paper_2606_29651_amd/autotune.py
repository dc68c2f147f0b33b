"""Autotuner for the work-class parameters (bin thresholds and the heavy 4-cycle
range) of niorca_count / niorca_count_batched.

A tuning run times each candidate parameter set on a representative workload
(median of a few calls) and keeps the fastest.  Results are stored in a text
file of "key name value" lines keyed by a workload label, the format the library
reads itself (niorca_load_tuning), so a later run loads them instead of searching
again.  Counts never depend on these parameters; only which kernel shape handles a
vertex does.
"""
from __future__ import annotations

import itertools
import os
import time
from typing import Callable, Dict, Iterable, List

DEFAULTS = {"tri_wave": 64, "tri_block": 480, "ql_wave": 512, "ql_block": 8192, "ql_split": 2048,
            "qh_wave": 512, "qh_block": 2048, "heavy_k": -1, "bin_mode": 0, "bin_deg_thread": 0,
            "bin_deg_group": 32, "bin_deg_block": 1 << 30}


def grid(**axes) -> List[Dict[str, int]]:
    """All combinations of the given parameter axes."""
    keys = list(axes)
    return [dict(zip(keys, vals)) for vals in itertools.product(*(axes[k] for k in keys))]


def apply(ctx, params: Dict[str, int]) -> None:
    for k, v in {**DEFAULTS, **params}.items():
        ctx.set_param(k, int(v))


def tune(ctx, run: Callable[[], None], candidates: Iterable[Dict[str, int]], repeats: int = 3,
         log: Callable[[str], None] = None) -> Dict:
    """Time run() under every candidate (after one warm-up call) and return
    {"best": params, "ms": best median ms, "table": [[params, ms], ...]}."""
    import torch
    table = []
    for cand in candidates:
        apply(ctx, cand)
        run()
        torch.cuda.synchronize()
        times = []
        for _ in range(repeats):
            t0 = time.perf_counter()
            run()
            torch.cuda.synchronize()
            times.append(1000.0 * (time.perf_counter() - t0))
        times.sort()
        ms = times[len(times) // 2]
        table.append([cand, ms])
        if log:
            log(f"[autotune] {cand} -> {ms:.3f} ms")
    best = min(table, key=lambda r: r[1])
    apply(ctx, best[0])
    return {"best": best[0], "ms": best[1], "table": table}


def save(path: str, key: str, params: Dict[str, int], note: str = "") -> None:
    """Replace the lines of `key` in the tuning file with params (other keys stay)."""
    keep = []
    if os.path.exists(path):
        with open(path) as f:
            keep = [ln for ln in f if not (ln.split() and ln.split()[0] == key)]
    lines = [f"{key} {name} {int(v)}" + (f"  # {note}" if note and i == 0 else "") + "\n"
             for i, (name, v) in enumerate(sorted(params.items()))]
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        f.writelines(keep + lines)
    os.replace(tmp, path)


def load(path: str, key: str):
    """{name: value} stored under key, or None."""
    if not os.path.exists(path):
        return None
    out = {}
    with open(path) as f:
        for ln in f:
            p = ln.split("#")[0].split()
            if len(p) == 3 and p[0] == key:
                out[p[1]] = int(p[2])
    return out or None
