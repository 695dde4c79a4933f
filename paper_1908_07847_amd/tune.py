"""Autotuner for libmlp launch shapes.

Choices tuned through `mlp_set_launch_hint` (include/mlp.h):

  * small / batched trainer, per size group: the waves of a net splitting
    its rows (128, 256 or 512 threads: more waves shorten one net's epoch,
    fewer let more nets share a CU) or its hidden layer (64: one wave per 16
    hidden units, one barrier per epoch and no per-wave partial gradients;
    best for the wide nets, which then fit three to a CU); and, for a plan
    of more than four groups, the side stream each group after the fourth
    follows (the group it waits for).
  * large-N trainer: the Gi x Gj grid (row blocks x hidden blocks) and the
    waves per workgroup (4 or 8).  More row blocks spread the minibatch wider
    but add partial gradients to sum; more hidden blocks shrink each
    workgroup's tile but add the cross-block output exchange; 8 waves (two
    per SIMD) overlap one wave's matrix-core work with another's vector work
    but halve each wave's registers.

Each candidate is timed on the caller's own data for a short run (HIP
events on the current stream) and the fastest is cached in a JSON file
(`$MLP_TUNE_CACHE`, default `~/.cache/paper_1908_07847_amd/tune.json`)
under a key of the device name, the workload kind and its shape buckets.
Results differ between launch shapes only in floating-point summation
order; for a fixed shape every run is bitwise repeatable, so a cached
choice also pins the bits.
"""
from __future__ import annotations

import json
import os
import time

import torch

from . import mlp
from ._lib import MLPError

CACHE_ENV = "MLP_TUNE_CACHE"
SMALL_CHOICES = (64, 128, 256, 512)   # 64: the hidden-split form


def cache_path() -> str:
    return os.environ.get(CACHE_ENV) or os.path.join(os.path.expanduser("~"), ".cache",
                                                     "paper_1908_07847_amd", "tune.json")


def _load_cache() -> dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(key: str, value) -> None:
    c = _load_cache()
    c[key] = value
    p = cache_path()
    os.makedirs(os.path.dirname(p), exist_ok=True)
    tmp = p + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(c, f, indent=1, sort_keys=True)
    os.replace(tmp, p)


def _device() -> str:
    return torch.cuda.get_device_name() if torch.cuda.is_available() else "cpu"


def _bucket(v: int) -> int:
    """Power-of-two bucket (shapes within a factor of two share a choice)."""
    b = 1
    while b < v:
        b *= 2
    return b


def small_key(n_in: int, max_rows: int, max_hidden: int, n_nets: int) -> str:
    return f"{_device()}|small|D{n_in}|N{_bucket(max_rows)}|H{_bucket(max_hidden)}|nets{_bucket(n_nets)}"


def large_key(n_in: int, n_hidden: int, batch: int, prec: str) -> str:
    return f"{_device()}|large|D{n_in}|H{_bucket(n_hidden)}|b{_bucket(batch)}|{prec}"


def large_candidates(n_hidden: int, batch: int, n_cu: int):
    """(Gi, Gj) grids the large trainer accepts for this shape: hidden blocks
    of 64..256 units and row blocks of >= 32 rows, one workgroup per CU."""
    out = []
    gj = 1
    while gj <= 16:
        hb = -(-n_hidden // (64 * gj)) * 64
        if 64 <= hb <= 256 or (gj == 1 and hb <= 256):
            gi = 1
            while gi * gj <= n_cu and gi <= 256:
                if batch % gi == 0 and (batch // gi) % 32 == 0:
                    out.append((gi, gj))
                gi *= 2
        gj *= 2
    return out


def _time(fn, reps: int = 2) -> float:
    fn()
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        s = torch.cuda.current_stream()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(s)
        fn()
        b.record(s)
        torch.cuda.synchronize()
        best = min(best, a.elapsed_time(b))
    return best


def tune_batched(plan: "mlp.BatchPlan", X, T, theta, n_in: int, n_out: int, epochs: int = 20,
                 force: bool = False, plan_epochs: int | None = None) -> list:
    """Pick threads per net for each group of the plan (mlp_train_batched
    launches; theta is not modified: candidates train copies), store them in
    plan.threads and return them.  Each group alone is timed for `epochs`
    epochs, the whole plan for `plan_epochs` (default `epochs`): plans that
    differ by a percent or two need the longer run to be told apart."""
    chosen = []
    for g, (start, count, max_rows, max_hidden) in enumerate(plan.groups):
        key = small_key(n_in, max_rows, max_hidden, count)
        cached = _load_cache().get(key)
        if cached and not force:
            chosen.append(int(cached["threads"]))
            continue
        times = {}
        saved = list(plan.threads)
        for t in SMALL_CHOICES:
            plan.threads[g] = t
            th = theta.clone()
            comp = torch.zeros_like(th)
            times[t] = _time(lambda: mlp.train_batched(plan, X, T, th, comp, epochs, n_in, n_out, groups=[g]))
        plan.threads[:] = saved
        best = min(times, key=times.get)
        _store(key, {"threads": best, "ms": times, "epochs": epochs, "when": time.time()})
        chosen.append(best)
    plan.threads[:] = chosen
    if len(plan.groups) > 1:
        chosen = _tune_together(plan, X, T, theta, n_in, n_out, plan_epochs or epochs, force)
    return chosen


def plan_key(n_in: int, plan: "mlp.BatchPlan") -> str:
    sig = ",".join(f"N{_bucket(r)}H{_bucket(h)}n{_bucket(c)}" for _, c, r, h in plan.groups)
    return f"{_device()}|smallplan|D{n_in}|{sig}"


def _tune_together(plan, X, T, theta, n_in, n_out, epochs, force):
    """The groups of a plan run concurrently, so a group's best shape alone
    need not be its best in company (a shape whose workgroups need a whole
    CU's LDS waits for CUs that the other groups keep busy).  Coordinate
    descent on the time of the whole plan: one pass over the groups' shapes
    (each trying every choice with the others fixed), one over the streams
    of the groups after the fourth, and, if a group moved, the shapes
    again."""
    key = plan_key(n_in, plan)
    cached = _load_cache().get(key)
    if cached and not force and len(cached["threads"]) == len(plan.groups):
        plan.threads[:] = [int(t) for t in cached["threads"]]
        if len(cached.get("streams", [])) == len(plan.groups):
            plan.stream_of[:] = [int(v) for v in cached["streams"]]
        return list(plan.threads)

    def whole():
        th = theta.clone()
        comp = torch.zeros_like(th)
        return _time(lambda: mlp.train_batched(plan, X, T, th, comp, epochs, n_in, n_out))

    best_t = whole()

    def threads_pass():
        nonlocal best_t
        for g in range(len(plan.groups)):
            keep = plan.threads[g]
            for t in SMALL_CHOICES:
                if t == keep:
                    continue
                plan.threads[g] = t
                tt = whole()
                if tt < best_t:
                    best_t, keep = tt, t
            plan.threads[g] = keep

    threads_pass()
    # a group after the fourth waits on its stream for the one before it
    # there: it should follow one that ends early, which the groups' costs
    # alone do not tell (a group of large workgroups is starved in company)
    moved = False
    for g in range(4, len(plan.groups)):
        keep = plan.stream_of[g]
        for v in range(4):
            if v == keep:
                continue
            plan.stream_of[g] = v
            tt = whole()
            if tt < best_t:
                best_t, keep, moved = tt, v, True
        plan.stream_of[g] = keep
    if moved:
        threads_pass()   # a group's best shape depends on its company
    _store(key, {"threads": list(plan.threads), "streams": list(plan.stream_of), "ms": best_t, "epochs": epochs,
                 "when": time.time()})
    return list(plan.threads)


def tune_large(n_in: int, n_hidden: int, n_out: int, batch: int, prec: str, X, T, theta,
               steps: int = 8, force: bool = False):
    """Pick the Gi x Gj grid and the waves per workgroup of the large-N
    trainer by timing `steps` minibatches of the caller's data (parameters
    are copied, not modified).  Returns (Gi, Gj, waves)."""
    key = large_key(n_in, n_hidden, batch, prec)
    cached = _load_cache().get(key)
    if cached and not force and "waves" in cached:
        return tuple(cached["grid"]) + (int(cached["waves"]),)
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    rows = min(X.shape[0], steps * batch)
    Xs, Ts = X[:rows], T[:rows]
    times = {}
    for grid in large_candidates(n_hidden, batch, n_cu):
        for waves in (4, 8):
            mlp.set_launch_hint(large_grid=grid, large_waves=waves)
            try:
                net = mlp.Net(n_in, n_hidden, n_out, rows, batch=batch, prec=prec, theta=theta)
                times[grid + (waves,)] = _time(lambda: net.train(Xs, Ts, 1, record_loss=False))
            except MLPError:
                continue
            finally:
                mlp.reset_launch_hint()
    best = min(times, key=times.get)
    _store(key, {"grid": list(best[:2]), "waves": best[2],
                 "ms": {f"{g[0]}x{g[1]}x{g[2]}": v for g, v in times.items()},
                 "steps": rows // batch, "when": time.time()})
    return best


def apply_small(n_in: int, max_rows: int, max_hidden: int, n_nets: int) -> bool:
    """Set the cached threads-per-net hint for this shape, if any."""
    c = _load_cache().get(small_key(n_in, max_rows, max_hidden, n_nets))
    if c:
        mlp.set_launch_hint(small_threads=int(c["threads"]))
        return True
    return False


def apply_batched(plan: "mlp.BatchPlan", n_in: int) -> bool:
    """Set plan.threads from the cache for every group that has an entry."""
    hit = False
    for g, (start, count, max_rows, max_hidden) in enumerate(plan.groups):
        c = _load_cache().get(small_key(n_in, max_rows, max_hidden, count))
        if c:
            plan.threads[g] = int(c["threads"])
            hit = True
    return hit


def apply_large(n_in: int, n_hidden: int, batch: int, prec: str) -> bool:
    """Set the cached grid hint for this shape, if any."""
    c = _load_cache().get(large_key(n_in, n_hidden, batch, prec))
    if c:
        mlp.set_launch_hint(large_grid=tuple(c["grid"]), large_waves=int(c.get("waves", 0)))
        return True
    return False
