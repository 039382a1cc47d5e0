"""Launch-shape autotuner for the force kernel.

For one precision and system size it times nbody_forces on random active
subsets of every size bucket 2^b and picks, per bucket, the number of
i thread-slots per workgroup (the rest of the 256 lanes split j inside the
workgroup) and the work-item target of the j-split; the kernel variant (one
or two i-particles per slot, j staged through LDS or broadcast from scalar
registers) is chosen on the full evaluation.  Results are
cached as JSON keyed by device architecture, precision and log2(N).

Every candidate computes the same sums in a different order, so tuning only
changes rounding (the split-invariance GPU test bounds the difference).

Usage: python -m paper_0909_0879_amd.autotune --n 1048576 --precision mixed
"""
from __future__ import annotations

import argparse
import json
import math
import os
import time

import numpy as np

from . import binding, ics

DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_cache.json")
SLOT_CHOICES = (1, 4, 16, 64, 256)
TARGET_CHOICES = (256, 1024, 2048, 4096, 8192)


def arch_name() -> str:
    import torch
    props = torch.cuda.get_device_properties(0)
    return getattr(props, "gcnArchName", "unknown").split(":")[0]


def cache_key(precision: int, n: int) -> str:
    return f"{arch_name()}/{'mixed' if precision == binding.MIXED else 'fp64'}/{int(round(math.log2(max(n, 1))))}"


def _time_forces(g, xt, vt, mt, ia, reps, acc_only=False):
    import torch
    call = (lambda: g.accel(xt, mt, i_active=ia)) if acc_only else \
        (lambda: g.forces(xt, vt, mt, i_active=ia))
    call()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        call()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def tune(n: int, precision: int, eps: float = 1e-3, seed: int = 77, buckets=None,
         verbose: bool = True, start: dict | None = None) -> dict:
    """Measure and return a tuning dict (the nbody_tuning fields).  Buckets
    not measured keep their values from start (else the library defaults)."""
    import torch
    m, x, v = ics.plummer(n, seed)
    xt, vt, mt = (torch.as_tensor(a, device="cuda") for a in (x, v, m))
    rng = np.random.default_rng(seed)
    top = int(math.floor(math.log2(n)))
    if buckets is None:
        buckets = list(range(0, top + 1))
    g = binding.NBody(m, x, v, eps=eps, precision=precision)
    base = dict(start) if start else g.get_tuning()
    # 1. kernel variant on the full evaluation
    full = torch.arange(n, dtype=torch.int32, device="cuda")
    # two interleaved rounds, best of each: box-to-box and run-to-run drift
    # is a few per cent, about the size of the differences being measured
    variants = (binding.VARIANT_K1, binding.VARIANT_K2, binding.VARIANT_S1, binding.VARIANT_S2)
    times = {var: math.inf for var in variants}
    for _ in range(2):
        for var in variants:
            g.set_tuning({"variant": var})
            times[var] = min(times[var], _time_forces(g, xt, vt, mt, full, 2))
    for var in variants:
        if verbose:
            print(f"variant {var}: full evaluation {times[var]:.2f} ms", flush=True)
    best_var = min(variants, key=lambda var: times[var])
    # the acceleration-only kernels (symplectic drivers, nbody_accel) carry
    # fewer registers and may prefer another variant
    acc_times = {var: math.inf for var in variants}
    for _ in range(2):
        for var in variants:
            g.set_tuning({"acc_variant": var})
            acc_times[var] = min(acc_times[var], _time_forces(g, xt, vt, mt, full, 2, True))
    for var in variants:
        if verbose:
            print(f"acc_variant {var}: full acceleration-only evaluation {acc_times[var]:.2f} ms",
                  flush=True)
    best_acc = min(variants, key=lambda var: acc_times[var])
    g.set_tuning({"acc_variant": -1})
    K = 2 if best_var in (binding.VARIANT_K2, binding.VARIANT_S2) else 1
    slots = list(base["i_slots"])
    targets = list(base["target_items"])
    # 2. per bucket: i-slots and split target
    for b in buckets:
        na = 1 << b
        ia = torch.as_tensor(np.sort(rng.choice(n, na, replace=False)).astype(np.int32),
                             device="cuda")
        reps = 20 if na * n < 1e9 else 3
        best = (math.inf, slots[b], targets[b])
        for s in SLOT_CHOICES:
            if s * K > 2 * na and s > 1:
                continue
            # on large systems thousands of active particles fill the chip
            # with full-width i-tiles and narrower ones only cost time to
            # try; on smaller ones the partial-row bound caps the j-splits
            # and narrower tiles are how the items reach the target
            if na >= 4096 and n >= (1 << 19) and s < 256:
                continue
            for tg in TARGET_CHOICES:
                tr = {"variant": best_var, "i_slots": [s] * binding.TUNE_BUCKETS,
                      "target_items": [tg] * binding.TUNE_BUCKETS}
                g.set_tuning(tr)
                t = _time_forces(g, xt, vt, mt, ia, reps)
                if verbose and na * n >= 1e11:
                    print(f"  bucket {b:2d}: slots {s:3d} target {tg:5d} {t:.3f} ms", flush=True)
                if t < best[0]:
                    best = (t, s, tg)
        slots[b], targets[b] = best[1], best[2]
        if verbose:
            rate = na * n / (best[0] * 1e-3)
            print(f"bucket {b:2d} (n_active {na}): slots {best[1]:3d} target {best[2]:5d} "
                  f"{best[0]:.3f} ms  {rate:.3e} int/s", flush=True)
    g.close()
    return {"variant": best_var, "acc_variant": best_acc, "use_graph": binding.GRAPH_ON,
            "steps_per_launch": 16,
            "min_split_j": 256, "i_slots": slots, "target_items": targets,
            "measured": time.strftime("%Y-%m-%dT%H:%M:%S")}


def load(precision: int, n: int, path: str = DEFAULT_CACHE):
    """Cached tuning for (arch, precision, log2 n), or None."""
    if not os.path.exists(path):
        return None
    with open(path) as f:
        cache = json.load(f)
    return cache.get(cache_key(precision, n))


def store(precision: int, n: int, tuning: dict, path: str = DEFAULT_CACHE):
    cache = {}
    if os.path.exists(path):
        with open(path) as f:
            cache = json.load(f)
    cache[cache_key(precision, n)] = tuning
    with open(path, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=1 << 20)
    ap.add_argument("--precision", choices=("fp64", "mixed"), default="mixed")
    ap.add_argument("--cache", default=DEFAULT_CACHE)
    ap.add_argument("--buckets", default="",
                    help="comma list of log2(n_active) buckets, or 'none' to choose only the "
                         "kernel variant (other buckets keep their cached values)")
    a = ap.parse_args()
    prec = binding.MIXED if a.precision == "mixed" else binding.FP64
    if a.buckets == "none":
        buckets = []
    else:
        buckets = [int(b) for b in a.buckets.split(",")] if a.buckets else None
    t = tune(a.n, prec, buckets=buckets, start=load(prec, a.n, a.cache))
    store(prec, a.n, t, a.cache)
    print(json.dumps({"key": cache_key(prec, a.n), **t}))


if __name__ == "__main__":
    main()
