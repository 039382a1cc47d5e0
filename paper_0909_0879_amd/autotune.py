"""Launch-shape autotuner for the force kernel.

For one precision and system size it times nbody_forces on random active
subsets of every size bucket 2^b and picks, per bucket, the number of
i thread-slots per workgroup (the rest of the 256 lanes split j inside the
workgroup) and the work-item target of the j-split; the kernel variant (one
or two i-particles per slot, j staged through LDS or broadcast from scalar
registers) is chosen on the full evaluation.  Results are
cached as JSON keyed by device architecture, precision and log2(N).

Ensembles of many clusters are tuned apart (--ensemble C): a block step of
an ensemble spreads over every cluster, so its time is set by the longest
work items, and narrower i-tiles than a single system of the same total N
wants pay off.  The ensemble tuner starts from the single-system entry of
the same size, caps the i-slots of the larger buckets, and times real block
steps of a seeded ensemble of Plummer clusters for each cap; then it widens
the i-tiles of the small buckets to their active counts (one work item per
j-split then serves all of a cluster's active particles, so each j tile is
predicted once for all of them, where the single-system entry spread a few
active particles over many items of a far longer j range) and searches the
smallest j-split.

Every candidate computes the same sums in a different order, so tuning only
changes rounding (the split-invariance GPU test bounds the difference).

Usage: python -m paper_0909_0879_amd.autotune --n 1048576 --precision mixed
       python -m paper_0909_0879_amd.autotune --ensemble 256 --precision mixed
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
TARGET_CHOICES = (256, 1024, 2048, 4096, 8192, 32768, 131072)


def arch_name() -> str:
    import torch
    props = torch.cuda.get_device_properties(0)
    return getattr(props, "gcnArchName", "unknown").split(":")[0]


PRECISION_NAMES = {binding.FP64: "fp64", binding.MIXED: "mixed", binding.MIXED_DS: "mixedds"}


def cache_key(precision: int, n: int, ensemble: bool = False) -> str:
    key = f"{arch_name()}/{PRECISION_NAMES[precision]}/{int(round(math.log2(max(n, 1))))}"
    return key + "/ensemble" if ensemble else key


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


def _nearest(cache: dict, key: str):
    """The entry of key, else the one of the nearest size with the same
    architecture, precision and kind (the smaller size on a tie), or None."""
    if key in cache:
        return cache[key]
    parts = key.split("/")
    size, suffix = int(parts[2]), parts[3:]
    best = None
    for k, entry in cache.items():
        q = k.split("/")
        if q[:2] != parts[:2] or q[3:] != suffix or not q[2].isdigit():
            continue
        d = (abs(int(q[2]) - size), int(q[2]))
        if best is None or d < best[0]:
            best = (d, entry)
    return best[1] if best else None


def load(precision: int, n: int, path: str = DEFAULT_CACHE, n_clusters: int = 1):
    """Cached tuning for (arch, precision, log2 n) — the nearest tuned size
    when n itself was not tuned — or None.  Contexts of several clusters
    take the ensemble entry of exactly their size when there is one (an
    ensemble entry is tuned to its kind of ensemble and is not stretched to
    other sizes)."""
    if not os.path.exists(path):
        return None
    with open(path) as f:
        cache = json.load(f)
    if n_clusters > 1 and cache_key(precision, n, True) in cache:
        return cache[cache_key(precision, n, True)]
    return _nearest(cache, cache_key(precision, n))


def store(precision: int, n: int, tuning: dict, path: str = DEFAULT_CACHE,
          ensemble: bool = False):
    cache = {}
    if os.path.exists(path):
        with open(path) as f:
            cache = json.load(f)
    cache[cache_key(precision, n, ensemble)] = tuning
    with open(path, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)


def tune_ensemble(n_clusters: int, precision: int, n_min: int = 256, n_max: int = 16384,
                  seed: int = 5000, t_end: float = 1 / 32, verbose: bool = True,
                  path: str = DEFAULT_CACHE) -> tuple[int, dict]:
    """Tune block steps of an ensemble of n_clusters Plummer clusters with
    log-uniform sizes in [n_min, n_max]; returns (total N, tuning)."""
    import torch
    m, x, v, off = ics.ensemble(n_clusters, n_min, n_max, seed=seed)
    n = int(m.shape[0])
    base = load(precision, n, path)
    if base is None:
        g = binding.NBody(m[:64], x[:64], v[:64], precision=precision)
        base = g.get_tuning()
        g.close()
    base = {k: val for k, val in base.items() if k != "measured"}

    def run(tr):
        best = math.inf
        for _ in range(2):
            g = binding.NBody(m, x, v, eps=1e-3, precision=precision, eta=0.01, eta_start=0.01,
                              level_min=5, level_max=20, cluster_offsets=off, tuning=tr)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            g.step(t_end)
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
            g.close()
        return best

    best = (run(base), 256, 0)
    if verbose:
        print(f"ensemble n={n}: single-system tuning {best[0]:.3f} s", flush=True)
    for cap in (128, 64, 32):
        for first in (6, 8, 10):
            tr = dict(base)
            tr["i_slots"] = [min(s, cap) if b >= first else s
                             for b, s in enumerate(base["i_slots"])]
            t = run(tr)
            if verbose:
                print(f"  i-slots <= {cap:3d} from bucket {first:2d}: {t:.3f} s", flush=True)
            if t < best[0]:
                best = (t, cap, first)
    out = dict(base)
    out["i_slots"] = [min(s, best[1]) if b >= best[2] else s
                      for b, s in enumerate(base["i_slots"])]
    # small buckets: i-slots 2^b for buckets 0 .. top (top = -1: as they
    # are), and the smallest j-split
    best_s = (best[0], -1, out["min_split_j"])
    for top in (4, 7):
        for msj in (256, 384, 512, 768):
            tr = dict(out)
            tr["i_slots"] = [min(1 << b, 256) if b <= top else s
                             for b, s in enumerate(out["i_slots"])]
            tr["min_split_j"] = msj
            t = run(tr)
            if verbose:
                print(f"  small buckets 0..{top} covered, min split {msj}: {t:.3f} s", flush=True)
            if t < best_s[0]:
                best_s = (t, top, msj)
    out["i_slots"] = [min(1 << b, 256) if b <= best_s[1] else s
                      for b, s in enumerate(out["i_slots"])]
    out["min_split_j"] = best_s[2]
    out["ensemble"] = {"clusters": n_clusters, "n_min": n_min, "n_max": n_max,
                       "slot_cap": best[1], "from_bucket": best[2],
                       "small_cover_to": best_s[1], "seconds": best_s[0]}
    out["measured"] = time.strftime("%Y-%m-%dT%H:%M:%S")
    if verbose:
        print(f"ensemble n={n}: i-slots <= {best[1]} from bucket {best[2]}, {best[0]:.3f} s",
              flush=True)
    return n, out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=1 << 20)
    ap.add_argument("--precision", choices=("fp64", "mixed", "mixedds"), default="mixed")
    ap.add_argument("--cache", default=DEFAULT_CACHE)
    ap.add_argument("--ensemble", type=int, default=0, metavar="C",
                    help="tune block steps of an ensemble of C Plummer clusters instead")
    ap.add_argument("--buckets", default="",
                    help="comma list of log2(n_active) buckets, or 'none' to choose only the "
                         "kernel variant (other buckets keep their cached values)")
    a = ap.parse_args()
    prec = {v: k for k, v in PRECISION_NAMES.items()}[a.precision]
    if a.ensemble > 1:
        n, t = tune_ensemble(a.ensemble, prec, path=a.cache)
        store(prec, n, t, a.cache, ensemble=True)
        print(json.dumps({"key": cache_key(prec, n, True), **t}))
        return
    if a.buckets == "none":
        buckets = []
    else:
        buckets = [int(b) for b in a.buckets.split(",")] if a.buckets else None
    t = tune(a.n, prec, buckets=buckets, start=load(prec, a.n, a.cache))
    store(prec, a.n, t, a.cache)
    print(json.dumps({"key": cache_key(prec, a.n), **t}))


if __name__ == "__main__":
    main()
