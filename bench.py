"""Training throughput of the one-hidden-layer sigmoid MLP trainer on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload w5] [--prec fp32]

The metric is training samples*epochs/s: rows processed by full training
steps (forward, error, backpropagation, gradient-descent update; arxiv
1908.07847 section 2.2) per second, with inputs already resident in HBM.

Default (the headline): w5 in float32 -- N = 4,194,304 rows x 64 features, a
64-1024-3 net, minibatches of 16384 rows (256 per epoch), K epochs (default
5).  A step is one epoch, run as one launch of the persistent trainer (the
launches continue one training run: parameters and the compensation carry
over); W untimed launches of one epoch come first.  The same K epochs are
then timed in the bf16 and e4m3 operand forms (field `forms`, each with
`vs_plain` = its rate over the float32 run); `--forms none` skips them.

Workloads (all synthetic, from the seeded generator):
  w1   60 rows x 33 features, 33-10-3 net, full batch           step = 1 epoch
  w2   120 rows x 33 features, 33-16-3 net, full batch           step = 1 epoch
  w3   4096 independent nets, H~U{4..64}, 40..120 rows each    step = 1 epoch of every net
  w4   1,048,576 x 33, 33-256-3, minibatch 4096               step = 1 epoch (256 minibatches)
  w5   4,194,304 x 64, 64-1024-3, minibatch 16384 (default)   step = 1 epoch (256 minibatches)
  w6   64 nets of w5's shape sharing its X (grid of 8 learning rates x 8 initialisations)
                                                               step = 1 epoch of every net
  w2d  w2's rows through a network with two hidden layers (33-16-16-3), every
       epoch in one launch (mlp_deep_train)            step = 1 epoch
  w2a  w2 through the differentiation path: per epoch MLPFunction (forward
       kernel), torch's MSE, the hand-written adjoint (backward kernels) and
       mlp_step, launched from Python                 step = 1 epoch
  p4   class predictions (mlp_predict: forward pass + argmax + correct count) on
       w4's 1,048,576 rows with its 33-256-3 net     metric: predicted rows/s
w4/w5 take --prec fp32|bf16|e4m3, w6 fp32|bf16 (operand precision of the two contractions).
The JSON line carries the roofline of the timed kernel (HIP events on the
stream it runs on; flops per launch are the method's algorithmic flops,
4DH + 6HK + 7H + 11K per sample-epoch plus 2P per update), the HBM bytes the
profiler counted for one launch (`traffic`, while the kernel source matches
the counters' record) and the FP64 CPU oracle's throughput on a bounded
sample of the same workload on the host cores (`cpu_baseline`).  w1-w3 also
report `repeats` and `vs_plain` (the chosen form against the plain
single-network FP32 kernel on the same GPU).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks (dense): fp32 vector/matrix 157.3 TFLOP/s, bf16 2.5
# PFLOP/s, fp8 5.0 PFLOP/s, HBM 8 TB/s.
PEAK = {"fp32": 157.3, "bf16": 2516.6, "e4m3": 5033.2}
PEAK_HBM_GBS = 8000.0


# Source files that define each timed kernel: a counter record in
# profiles/counters.json applies only while these are unchanged.
KERNEL_SOURCES = {
    "small": ["small_train.hip", "mlp_device.hpp"],
    "large": ["large_train.hip", "mlp_device.hpp", "mlp_large.hpp"],
    "layer": ["layer.hip", "mlp_device.hpp"],
}


def kernel_source_hash(kind: str) -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kind]:
        with open(os.path.join(ROOT, "paper_1908_07847_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(key: str, kind: str):
    """HBM bytes per launch from the profiler's FETCH_SIZE and WRITE_SIZE
    counters (scaled by a plain copy of known size), if a record for this
    workload was taken on the current kernel source; else None."""
    try:
        with open(os.path.join(ROOT, "profiles", "counters.json")) as f:
            rec = json.load(f)[key]
    except (OSError, ValueError, KeyError):
        return None
    if rec.get("source") != kernel_source_hash(kind):
        return None
    return rec["hbm_bytes_per_launch"]


def measured_traffic_per_epoch(key: str, kind: str):
    """HBM bytes of one launch of one epoch (FETCH_SIZE + WRITE_SIZE, each
    scaled by a plain copy of known size) for a large workload, if a record
    taken on the current kernel source exists; else None."""
    try:
        with open(os.path.join(ROOT, "profiles", "counters.json")) as f:
            rec = json.load(f)[key]
    except (OSError, ValueError, KeyError):
        return None
    if rec.get("source") != kernel_source_hash(kind) or "hbm_bytes_per_epoch" not in rec:
        return None
    return rec["hbm_bytes_per_epoch"]


def counters_record(fetch_csv: str, write_csv: str, copy_fetch_csv: str, copy_write_csv: str, kernel_prefix: str,
                    copy_bytes: int = 1 << 30, kernel_dispatch: int = -1) -> dict:
    """HBM bytes of one dispatch from rocprofv3 --pmc counter files.

    FETCH_SIZE and WRITE_SIZE are read (KiB per dispatch, summed over the
    counter's instances) for the dispatch of `kernel_prefix` numbered
    `kernel_dispatch` among that kernel's dispatches (default: the last),
    and each is scaled by the factor that turns the same counter's reading
    for a plain device copy of `copy_bytes` bytes into the bytes that copy
    moves (the copy reads and writes `copy_bytes` each)."""
    import csv

    def per_dispatch(path, name_match):
        vals = {}
        with open(path) as f:
            for row in csv.DictReader(f):
                if not name_match(row["Kernel_Name"]):
                    continue
                d = int(row["Dispatch_Id"])
                vals[d] = vals.get(d, 0.0) + float(row["Counter_Value"])
        return [vals[k] for k in sorted(vals)]

    def is_copy(n):
        return "copy" in n.lower() or "elementwise" in n.lower()

    def is_kernel(n):
        return n.startswith(kernel_prefix)

    cf = max(per_dispatch(copy_fetch_csv, is_copy))
    cw = max(per_dispatch(copy_write_csv, is_copy))
    f_scale = copy_bytes / (cf * 1024.0)
    w_scale = copy_bytes / (cw * 1024.0)
    kf = per_dispatch(fetch_csv, is_kernel)[kernel_dispatch]
    kw = per_dispatch(write_csv, is_kernel)[kernel_dispatch]
    return {"fetch_kib": kf, "write_kib": kw, "fetch_scale": f_scale, "write_scale": w_scale,
            "hbm_bytes": kf * 1024.0 * f_scale + kw * 1024.0 * w_scale}


def flops_per_sample_epoch(D: int, H: int, K: int) -> int:
    """Algorithmic flops of one sample through one training step.

    forward  2DH (z1 = b1 + sum x w) + 3H (sigmoid: negate, add 1, divide) + 2HK + 3K
    error    3K (difference, square, accumulate)
    deltas   4K (delta2 = c e y (1-y)) + 2HK (delta2 W2) + 3H (times a (1-a))
    grads    2DH + H (gW1, gb1) + 2HK + K (gW2, gb2)
    total    4DH + 6HK + 7H + 11K, plus H + K exponentials counted separately.
    The update adds 2P flops per step, P = DH + H + HK + K.
    """
    return 4 * D * H + 6 * H * K + 7 * H + 11 * K


def cpu_info() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def timed(fn, stream):
    import torch
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    fn()
    ev1.record(stream)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, ev0.elapsed_time(ev1) / 1e3


# grid-wide synchronisations per minibatch step of the large-N trainer
LARGE_BARRIERS_PER_STEP = 3


def sync_adjusted(mlp, torch, flops: float, peak_tflops: float, hbm_bytes: float, n_steps: int, kernel_s: float):
    """The sync-adjusted bound for the persistent large-N trainer:
    max(flops / peak, bytes / HBM bandwidth) plus, per minibatch step, its
    grid barriers at the latency measured on this GPU (mlp_barrier_probe with
    one workgroup per CU, the grid the trainer's plans use here)."""
    n_wg = torch.cuda.get_device_properties(0).multi_processor_count
    t_bar = mlp.barrier_latency_us(n_wg)
    nb = LARGE_BARRIERS_PER_STEP
    bound_s = max(flops / (peak_tflops * 1e12), hbm_bytes / (PEAK_HBM_GBS * 1e9)) + n_steps * nb * t_bar * 1e-6
    return {"t_barrier_us": t_bar, "barriers_per_step": nb, "steps": n_steps, "workgroups": n_wg,
            "bound_ms": bound_s * 1e3, "frac": bound_s / kernel_s}


def repeats(fn, stream, first_wall: float, steps: int, max_wall: float = 1.5, runs: int = 5):
    """Median and minimum over the timed run and up to `runs` more runs of
    the same K steps (only when one run is short)."""
    ms = [first_wall * 1e3 / steps]
    if first_wall < max_wall:
        for _ in range(runs):
            ms.append(timed(fn, stream)[0] * 1e3 / steps)
    return {"runs": len(ms), "median_ms_per_step": float(np.median(ms)), "min_ms_per_step": float(min(ms))}


# ---------------------------------------------------------------- single nets (w1, w2, w4, w5)
def bench_single(args):
    import torch
    from paper_1908_07847_amd import mlp, synth

    wl = int(args.workload[1])
    w = synth.single(wl)
    D, H, K, N = w["D"], w["H"], w["K"], w["X"].shape[0]
    batch = w["batch"] or N
    prec = "fp32"
    act, mu = args.act, args.momentum
    net = mlp.Net(D, H, K, N, batch=w["batch"], lr=w["lr"], prec=prec, theta=w["theta"], act=act, momentum=mu)
    X = torch.from_numpy(w["X"]).cuda()
    T = torch.from_numpy(w["T"]).cuda()
    steps = args.steps if args.steps is not None else w["epochs"]
    warmup = args.warmup if args.warmup is not None else (100 if wl <= 2 else 1)
    hist = torch.empty(max(steps, warmup, 1), device="cuda")
    if warmup:
        net.train(X, T, warmup, loss_hist=hist[:warmup])
    stream = torch.cuda.current_stream()
    wall, kern = timed(lambda: net.train(X, T, steps, loss_hist=hist[:steps]), stream)
    final_loss = float(hist[steps - 1].item()) if steps else None
    reps = repeats(lambda: net.train(X, T, steps, loss_hist=hist[:steps]), stream, wall, steps)
    vs_plain = None
    P = D * H + H + H * K + K
    n_updates = steps * (-(-N // batch))
    flops = flops_per_sample_epoch(D, H, K) * N * steps + 2 * P * n_updates
    bound, peak, unit, kname, kind = "alu", PEAK["fp32"], "TFLOP/s", "mlpk::k_small_train", "small"
    tkey = f"{args.workload}-{prec}-steps{steps}"
    achieved = flops / kern / 1e12
    names = {1: "plain-small: N=60 x 33, 33-10-3, full batch",
             2: "differentiation: N=120 x 33, 33-16-3, full batch (fused mlp_train)"}
    res = dict(
        metric="training samples*epochs/s", value=N * steps / wall, unit="samples*epochs/s",
        ms_per_step=wall * 1e3 / steps, dtype={"fp32": "f32", "bf16": "bf16", "e4m3": "e4m3"}[prec],
        config={"workload": names[wl] + (", sigmoid both layers" if act == "sigmoid" else
                                         ", tanh hidden / sigmoid output (variant)") + ", MSE, " +
                    ("GD lr=0.1" if not mu else f"heavy-ball momentum {mu}, lr={w['lr']} (variant)"), "n_rows": N, "n_in": D,
                "n_hidden": H, "n_out": K, "batch": batch, "lr": w["lr"], "compensated_update": True,
                "operand_precision": prec, "hidden_activation": act, "momentum": mu, "step": "one epoch"},
        roofline={"bound": bound, "achieved": achieved, "peak": peak, "unit": unit, "frac": achieved / peak,
                  "traffic": measured_traffic(tkey, kind), "traffic_unit": "bytes per launch", "kernel": kname,
                  "kernel_ms": kern * 1e3, "flops_per_launch": flops},
        final_loss=final_loss, repeats=reps, vs_plain=vs_plain, steps=steps, warmup=warmup)
    # one net is one workgroup on one of the 256 CUs: its honest denominator
    # is one CU's share of the FP32 rate, and the per-epoch latency
    cu_peak = PEAK["fp32"] / 256
    res["roofline"]["one_cu"] = {"peak": cu_peak, "unit": "TFLOP/s", "frac": achieved / cu_peak,
                                 "epoch_us": kern * 1e6 / steps}
    return res, dict(w=w, wl=wl, batch=batch, act=act, mu=mu)


def cpu_single(ctx, budget_s: float):
    import oracle
    w, wl, batch = ctx["w"], ctx["wl"], ctx["batch"]
    p = oracle.Params.of(w["theta"])
    X, T, epochs, rows = w["X"], w["T"], w["epochs"], w["X"].shape[0]
    sample = f"the full workload ({rows} rows x {epochs} epochs)"
    reps, t_total = 0, 0.0
    while (t_total < budget_s or reps == 0) and reps < 100000:
        t0 = time.perf_counter()
        if ctx.get("act", "sigmoid") != "sigmoid" or ctx.get("mu", 0.0):
            oracle.train_var(X, T, p, w["lr"], epochs, act=ctx["act"], mu=ctx["mu"])
        else:
            oracle.train(X, T, p, w["lr"], epochs, batch=0)
        t_total += time.perf_counter() - t0
        reps += 1
    return {"value": rows * epochs * reps / t_total, "unit": "samples*epochs/s", "cores": 1, "kind": "oracle",
            "sample": f"{sample}, run {reps} time(s), float64, single thread, {cpu_info()}",
            "seconds": t_total}


# ---------------------------------------------------------------- large N (w4, w5: the headline)
LARGE_NAMES = {4: "large-N: N=1,048,576 x 33, 33-256-3, minibatch 4096",
               5: "wide: N=4,194,304 x 64, 64-1024-3, minibatch 16384"}


def per_launch_times(launch, stream, count: int):
    """Run `launch(i)` for i < count back to back on `stream`; returns the
    wall time of the whole run and each launch's duration from HIP events
    recorded between the launches (on the stream the kernel runs on)."""
    import torch
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(count + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evs[0].record(stream)
    for i in range(count):
        launch(i)
        evs[i + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, [evs[i].elapsed_time(evs[i + 1]) / 1e3 for i in range(count)]


def large_form(mlp, torch, w, X, T, prec: str, steps: int, warmup: int):
    """One operand form of a large workload: `warmup` untimed launches, then
    `steps` timed launches of one epoch each (every launch runs the epoch's
    minibatch steps; parameters carry over, so the launches together are one
    training run of `steps` epochs).  Returns the numbers of the timed run."""
    D, H, K, N = w["D"], w["H"], w["K"], w["X"].shape[0]
    net = mlp.Net(D, H, K, N, batch=w["batch"], lr=w["lr"], prec=prec, theta=w["theta"])
    hist = torch.empty(max(steps, warmup, 1), device="cuda")
    for i in range(warmup):
        net.train(X, T, 1, loss_hist=hist[i:i + 1])
    net.set_theta(w["theta"])
    stream = torch.cuda.current_stream()
    wall, durs = per_launch_times(lambda i: net.train(X, T, 1, loss_hist=hist[i:i + 1]), stream, steps)
    out = dict(wall=wall, durs=durs, kernel_s=float(np.mean(durs)),
               final_loss=float(hist[steps - 1].item()) if steps else None)
    net.close()
    return out


def bench_large(args):
    import torch
    from paper_1908_07847_amd import mlp, synth

    wl = int(args.workload[1])
    w = synth.single(wl)
    D, H, K, N, batch = w["D"], w["H"], w["K"], w["X"].shape[0], w["batch"]
    X = torch.from_numpy(w["X"]).cuda()
    T = torch.from_numpy(w["T"]).cuda()
    steps = args.steps if args.steps is not None else w["epochs"]
    warmup = args.warmup if args.warmup is not None else 1
    P = D * H + H + H * K + K
    spe = -(-N // batch)                                      # minibatch steps per epoch
    F = flops_per_sample_epoch(D, H, K)
    flops_epoch = F * N + 2 * P * spe                         # one launch = one epoch
    prec = args.prec
    forms = [prec] + ([q for q in ("bf16", "e4m3") if q != prec] if args.forms == "all" else [])
    res_forms = {}
    for q in forms:
        r = large_form(mlp, torch, w, X, T, q, steps, warmup if q == prec else min(warmup, 1))
        ach = flops_epoch / r["kernel_s"] / 1e12
        res_forms[q] = dict(value=N * steps / r["wall"], ms_per_step=r["wall"] * 1e3 / steps,
                            kernel_ms_per_launch=r["kernel_s"] * 1e3,
                            median_ms_per_launch=float(np.median(r["durs"])) * 1e3,
                            min_ms_per_launch=float(min(r["durs"])) * 1e3,
                            kernel=mlp.large_plan(D, H, K, N, batch=batch, prec=q)["kernel"],
                            achieved_tflops=ach, peak_tflops=PEAK[q], frac=ach / PEAK[q],
                            final_loss=r["final_loss"], dtype={"fp32": "f32", "bf16": "bf16", "e4m3": "e4m3"}[q])
    head = res_forms[prec]
    for q in forms[1:]:
        res_forms[q]["vs_plain"] = res_forms[q]["value"] / res_forms["fp32"]["value"] if "fp32" in res_forms else None
    kern = head["kernel_ms_per_launch"] / 1e3
    tkey = f"{args.workload}-{prec}"
    per_epoch = measured_traffic_per_epoch(tkey, "large")
    res = dict(
        metric="training samples*epochs/s", value=head["value"], unit="samples*epochs/s",
        ms_per_step=head["ms_per_step"], dtype=head["dtype"],
        config={"workload": LARGE_NAMES[wl] + ", sigmoid both layers, MSE, GD lr=0.1, float32 master "
                            "parameters, compensated update", "n_rows": N, "n_in": D, "n_hidden": H, "n_out": K,
                "batch": batch, "lr": w["lr"], "operand_precision": prec,
                "step": f"one epoch ({spe} minibatch steps) = one launch of the persistent trainer"},
        roofline={"bound": "mfma", "achieved": head["achieved_tflops"], "peak": PEAK[prec], "unit": "TFLOP/s",
                  "frac": head["frac"], "traffic": per_epoch, "traffic_unit": "HBM bytes per launch (one epoch)",
                  "algorithmic_bytes": N * (D + K) * 4 + 2 * P * 4,
                  "kernel": head["kernel"], "kernel_ms": head["kernel_ms_per_launch"],
                  "flops_per_launch": flops_epoch,
                  "flops_per_sample_epoch": F, "update_flops_per_step": 2 * P},
        forms={q: v for q, v in res_forms.items() if q != prec},
        final_loss=head["final_loss"],
        repeats={"runs": steps, "median_ms_per_step": head["median_ms_per_launch"],
                 "min_ms_per_step": head["min_ms_per_launch"], "note": "per timed launch (HIP events)"},
        steps=steps, warmup=warmup)
    res["roofline"]["sync_adjusted"] = sync_adjusted(mlp, torch, flops_epoch, PEAK[prec], N * (D + K) * 4.0,
                                                     spe, kern)
    return res, dict(w=w, wl=wl, batch=batch)


def cpu_large(ctx, budget_s: float, rows: int = 65536):
    """The oracle (float64) trains on the first `rows` rows (whole minibatches)
    for one epoch, repeated until `budget_s` has passed, on every host core
    (its loops over gradient entries and rows are shared among OpenMP
    threads), from a timing build of the same sources (-O3 -march=native)."""
    import tempfile
    import oracle
    w, batch = ctx["w"], ctx["batch"]
    lib = oracle.build_timing(tempfile.mkdtemp(prefix="oracle_timing_"))
    p = oracle.Params.of(w["theta"])
    X, T = w["X"][:rows], w["T"][:rows]
    with oracle.use_library(lib):
        oracle.set_threads(0)
        threads = oracle.max_threads()
        reps, t_total = 0, 0.0
        while (t_total < budget_s or reps == 0) and reps < 100000:
            t0 = time.perf_counter()
            oracle.train(X, T, p, w["lr"], 1, batch=batch)
            t_total += time.perf_counter() - t0
            reps += 1
    return {"value": rows * reps / t_total, "unit": "samples*epochs/s", "cores": threads, "kind": "oracle",
            "sample": f"the first {rows} rows ({rows // batch} minibatches of {batch}) for 1 epoch, run {reps} "
                      f"time(s), float64, {threads} OpenMP threads, -O3 -march=native build, {cpu_info()}",
            "seconds": t_total}


# ---------------------------------------------------------------- batched (w3)
def bench_batched(args):
    import torch
    from paper_1908_07847_amd import mlp, synth, tune

    w = synth.batched(heldout=True)
    items = w["items"]
    plan = mlp.BatchPlan(items, buckets=not args.no_buckets)
    X = torch.from_numpy(w["X"]).cuda()
    T = torch.from_numpy(w["T"]).cuda()
    th = torch.from_numpy(w["theta"]).cuda()
    comp = torch.zeros_like(th)
    steps = args.steps if args.steps is not None else w["epochs"]
    warmup = args.warmup if args.warmup is not None else 5
    # launch shape of each size group from the autotuner (timed on copies,
    # cached per device and group shape)
    threads = tune.tune_batched(plan, X, T, th, 33, 3, epochs=100, plan_epochs=500)
    if warmup:
        mlp.train_batched(plan, X, T, th.clone(), torch.zeros_like(th), warmup, 33, 3)
    hist = torch.empty((len(items), steps), device="cuda")
    # the timed launch is one replay of a HIP graph holding the whole run
    graph = mlp.BatchedGraph(plan, X, T, th, comp, steps, 33, 3, loss_hist=hist)
    stream = torch.cuda.current_stream()
    wall, kern = timed(graph.replay, stream)
    reps = repeats(graph.replay, stream, wall, steps)
    # plain form: the single-network kernel launched once per net, one net
    # after another, on the first 32 nets
    sample = items[:32]
    nets = []
    for it in sample:
        H = it["n_hidden"]
        P = 33 * H + H + 3 * H + 3
        r0, n = it["x_off"], it["n_rows"]
        nets.append((mlp.Net(33, H, 3, n, lr=float(it["lr"]),
                             theta=synth.Theta.unpack(w["theta"][it["p_off"]:it["p_off"] + P], 33, H, 3)),
                     X[r0:r0 + n].clone(), T[r0:r0 + n].clone()))   # own (aligned) allocations
    for net, Xi, Ti in nets[:2]:
        net.train(Xi, Ti, 1)

    def plain_loop():
        for net, Xi, Ti in nets:
            net.train(Xi, Ti, steps)
    pwall, _ = timed(plain_loop, stream)
    prows = sum(it["n_rows"] for it in sample)
    vs_plain = {"speedup": (sum(it["n_rows"] for it in items) * steps / wall) / (prows * steps / pwall),
                "plain_value": prows * steps / pwall,
                "plain": "the single-network FP32 kernel, one launch per net, nets one after another",
                "sample": f"the first {len(sample)} nets, {steps} epochs each"}
    # cross-validation read-out: every net on its held-out fold (mlp_eval_batched),
    # then the hyperparameter group with the lowest mean held-out loss
    vplan = mlp.BatchPlan(w["items_val"])
    Xv, Tv = torch.from_numpy(w["X_val"]).cuda(), torch.from_numpy(w["T_val"]).cuda()
    mlp.eval_batched(vplan, Xv, Tv, th, 33, 3)
    _, eval_s = timed(lambda: mlp.eval_batched(vplan, Xv, Tv, th, 33, 3), stream)
    vloss, vcor = mlp.eval_batched(vplan, Xv, Tv, th, 33, 3)
    # the group (hidden size, learning rate) with the lowest mean held-out
    # loss over its folds, selected on the device
    groups = np.array([it["group"] for it in w["items_val"]])
    ng = int(groups.max()) + 1
    gmean_d, best_d = mlp.cv_select(vloss, torch.from_numpy(groups.astype(np.int32)).cuda(), ng)
    gmean, best = gmean_d.cpu().numpy(), int(best_d.item())
    vloss, vcor = vloss.cpu().numpy(), vcor.cpu().numpy()
    vrows = int(sum(it["n_rows"] for it in w["items_val"]))
    rows = sum(it["n_rows"] for it in items)
    flops = 0
    for it in items:
        H = it["n_hidden"]
        P = 33 * H + H + 3 * H + 3
        flops += (flops_per_sample_epoch(33, H, 3) * it["n_rows"] + 2 * P) * steps
    achieved = flops / kern / 1e12
    res = dict(
        metric="training samples*epochs/s", value=rows * steps / wall, unit="samples*epochs/s",
        ms_per_step=wall * 1e3 / steps, dtype="f32",
        config={"workload": "batched: 4096 independent 33-H-3 nets, H~U{4..64}, 40..120 rows each "
                            "(5-fold CV splits), lr~logU(0.01,1), full batch, one launch",
                "nets": len(items), "total_rows": rows, "step": "one epoch of every net",
                "threads_per_net": threads,
                "groups": [{"nets": c, "max_rows": r, "max_hidden": h, "stream": plan.stream_of[g]}
                           for g, (_, c, r, h) in enumerate(plan.groups)],
                "launch": "hipGraph replay of one trainer launch per size group"},
        cv_eval={"kernel": "mlpk::k_eval_batched + mlpk::k_cv_select", "ms": eval_s * 1e3, "heldout_rows": vrows,
                 "rows_per_s": vrows / eval_s, "best_group": best, "best_group_hidden": int(
                     w["items_val"][int(np.nonzero(groups == best)[0][0])]["n_hidden"]),
                 "best_mean_heldout_loss": float(gmean[best]),
                 "heldout_accuracy": float(vcor.sum() / vrows)},
        roofline={"bound": "alu", "achieved": achieved, "peak": PEAK["fp32"], "unit": "TFLOP/s",
                  "frac": achieved / PEAK["fp32"], "traffic": measured_traffic(f"w3-fp32-steps{steps}", "small"),
                  "traffic_unit": "bytes per launch",
                  "kernel": " + ".join(sorted({"mlpk::k_small_hsplit" if t == 64 else "mlpk::k_small_train"
                                               for t in threads})) + " (one launch per size group)",
                  "kernel_ms": kern * 1e3, "flops_per_launch": flops}, repeats=reps, vs_plain=vs_plain,
        steps=steps, warmup=warmup)
    return res, dict(w=w)


def cpu_batched(ctx, budget_s: float):
    import oracle
    w = ctx["w"]
    items = w["items"][:64]
    epochs = 100
    threads = oracle.max_threads()
    reps, t_total = 0, 0.0
    while (t_total < budget_s or reps == 0) and reps < 100000:
        t0 = time.perf_counter()
        oracle.train_many(items, w["X"], w["T"], w["theta"], 33, 3, epochs, threads=threads)
        t_total += time.perf_counter() - t0
        reps += 1
    rows = sum(it["n_rows"] for it in items)
    return {"value": rows * epochs * reps / t_total, "unit": "samples*epochs/s", "cores": threads,
            "kind": "oracle", "sample": f"the first 64 nets for {epochs} epochs, run {reps} time(s), float64, "
                                        f"one net per thread, {cpu_info()}", "seconds": t_total}


# ---------------------------------------------------------------- nets sharing X (w6)
def bench_shared(args):
    import torch
    from paper_1908_07847_amd import mlp, synth

    prec = args.prec if args.prec in ("fp32", "bf16") else "bf16"
    w = synth.shared(5, n_nets=64)
    D, H, K, N, batch = w["D"], w["H"], w["K"], w["X"].shape[0], w["batch"]
    M = w["theta"].shape[0]
    X = torch.from_numpy(w["X"]).cuda()
    T = torch.from_numpy(w["T"]).cuda()
    th0 = torch.from_numpy(w["theta"]).cuda()
    ws = torch.empty(mlp.shared_workspace_size(D, H, K, N, batch, M, prec), dtype=torch.uint8, device="cuda")
    steps = args.steps if args.steps is not None else w["epochs"]
    warmup = args.warmup if args.warmup is not None else 1
    if warmup:
        mlp.train_shared(X, T, th0.clone(), w["lrs"], warmup, H, batch=batch, prec=prec,
                         comp=torch.zeros_like(th0), workspace=ws)
    th, comp = th0.clone(), torch.zeros_like(th0)
    hist = torch.empty((M, max(steps, 1)), device="cuda")
    stream = torch.cuda.current_stream()
    wall, kern = timed(lambda: mlp.train_shared(X, T, th, w["lrs"], steps, H, batch=batch, prec=prec, comp=comp,
                                                loss_hist=hist[:, :steps], workspace=ws), stream)
    final_loss_mean = float(hist[:, steps - 1].mean().item()) if steps else None
    # plain form: one net of the same shape on the single-network FP32
    # kernel (the 64 nets would run one after another), one epoch
    plain = mlp.Net(D, H, K, N, batch=batch, lr=float(w["lrs"][0]), prec="fp32",
                    theta=synth.Theta.unpack(w["theta"][0], D, H, K))
    plain.train(X, T, 1)
    pwall, _ = timed(lambda: plain.train(X, T, 1), stream)
    vs_plain = {"speedup": (M * N * steps / wall) / (N / pwall), "plain_value": N / pwall,
                "plain": "one net of the same shape on the single-network FP32 kernel (the nets one after another)",
                "sample": "net 0, one epoch"}
    P = D * H + H + H * K + K
    flops = (flops_per_sample_epoch(D, H, K) * N + 2 * P * (-(-N // batch))) * M * steps
    achieved = flops / kern / 1e12
    res = dict(
        metric="training samples*epochs/s", value=M * N * steps / wall, unit="samples*epochs/s",
        ms_per_step=wall * 1e3 / steps, dtype={"fp32": "f32", "bf16": "bf16"}[prec],
        config={"workload": "64 nets sharing X: N=4,194,304 x 64, 64-1024-3 each, minibatch 16384, lr grid "
                            "10^(-2..0) x 8 initialisations, sigmoid both layers, MSE, GD, one launch",
                "nets": M, "n_rows": N, "n_in": D, "n_hidden": H, "n_out": K, "batch": batch,
                "compensated_update": True, "operand_precision": prec, "step": "one epoch of every net"},
        roofline={"bound": "mfma", "achieved": achieved, "peak": PEAK[prec], "unit": "TFLOP/s",
                  "frac": achieved / PEAK[prec], "traffic": measured_traffic(f"w6-{prec}-steps{steps}", "large"),
                  "traffic_unit": "bytes per launch",
                  "kernel": mlp.large_plan(D, H, K, N, batch=batch, prec=prec, n_nets=M)["kernel"],
                  "kernel_ms": kern * 1e3, "flops_per_launch": flops},
        final_loss_mean=final_loss_mean, repeats={"runs": 1, "median_ms_per_step": wall * 1e3 / steps,
                                                  "min_ms_per_step": wall * 1e3 / steps},
        vs_plain=vs_plain, steps=steps, warmup=warmup)
    res["roofline"]["sync_adjusted"] = sync_adjusted(mlp, torch, flops, PEAK[prec], N * steps * (D + K) * 4.0,
                                                     steps * (-(-N // batch)), kern)
    return res, dict(w=w, batch=batch)


def cpu_shared(ctx, budget_s: float):
    """The oracle trains net after net; one net on the first minibatch for
    one epoch is the sample (the nets are independent, so the rate of one
    thread on one net is the oracle's rate for the grid)."""
    import oracle
    from paper_1908_07847_amd import synth
    w, batch = ctx["w"], ctx["batch"]
    p = oracle.Params.of(synth.Theta.unpack(w["theta"][0], w["D"], w["H"], w["K"]))
    X, T = w["X"][:batch], w["T"][:batch]
    reps, t_total = 0, 0.0
    while (t_total < budget_s or reps == 0) and reps < 100000:
        t0 = time.perf_counter()
        oracle.train(X, T, p, w["lrs"][0], 1, batch=batch)
        t_total += time.perf_counter() - t0
        reps += 1
    return {"value": batch * reps / t_total, "unit": "samples*epochs/s", "cores": 1, "kind": "oracle",
            "sample": f"net 0 on the first {batch} rows (one minibatch) for 1 epoch, run {reps} time(s), "
                      f"float64, single thread, {cpu_info()}", "seconds": t_total}


# ---------------------------------------------------------------- several hidden layers (w2d)
DEEP_WIDTHS = [33, 16, 16, 3]


def bench_deep(args):
    import torch
    from paper_1908_07847_amd import mlp, synth

    w = synth.single(2)
    widths, N = DEEP_WIDTHS, w["X"].shape[0]
    theta = np.random.default_rng(2).uniform(-0.5, 0.5, mlp.deep_n_params(widths)).astype(np.float32)
    net = mlp.DeepNet(widths, theta=theta, act=args.act)
    X = torch.from_numpy(w["X"]).cuda()
    T = torch.from_numpy(w["T"]).cuda()
    steps = args.steps if args.steps is not None else 1000
    warmup = args.warmup if args.warmup is not None else 20
    G = 50   # epochs per captured graph
    if steps % G:
        raise SystemExit(f"w2d: --steps must be a multiple of {G}")
    hist = torch.empty(max(steps, warmup, 1), device="cuda")
    stream = torch.cuda.current_stream()
    # reference form: torch.autograd over DenseFunction, launched from Python
    net.train(X, T, warmup, loss_hist=hist)
    ag_epochs = min(steps, 200)
    awall, _ = timed(lambda: net.train(X, T, ag_epochs, loss_hist=hist), stream)
    # the per-layer library calls of one epoch replayed from a HIP graph of G epochs
    net.flat.detach().copy_(torch.from_numpy(theta))
    net.comp.zero_()
    graph = mlp.DeepGraph(net, X, T, G)

    def run_graph():
        for r in range(steps // G):
            graph.replay()
            hist[r * G:(r + 1) * G].copy_(graph.loss)
    gwall, _ = timed(run_graph, stream)
    # timed form: every epoch in one launch (mlp_deep_train)
    net.flat.detach().copy_(torch.from_numpy(theta))
    net.comp.zero_()
    net.train_kernel(X, T, warmup, loss_hist=hist)
    net.flat.detach().copy_(torch.from_numpy(theta))
    net.comp.zero_()
    wall, kern = timed(lambda: net.train_kernel(X, T, steps, loss_hist=hist), stream)
    final_loss = float(hist[steps - 1].item()) if steps else None
    reps = repeats(lambda: net.train_kernel(X, T, steps, loss_hist=hist), stream, wall, steps)
    # per sample-epoch: forward 2 w(l) w(l+1) + activation, backward 4 w(l) w(l+1) (gW and dX; dX skipped for
    # the first layer), plus the update 2P per epoch
    P = mlp.deep_n_params(widths)
    f = 0
    for l in range(len(widths) - 1):
        f += 2 * widths[l] * widths[l + 1] + 2 * widths[l] * widths[l + 1] + (2 * widths[l] * widths[l + 1] if l else 0)
        f += 4 * widths[l + 1]
    flops = f * N * steps + 2 * P * steps
    achieved = flops / kern / 1e12
    cu_peak = PEAK["fp32"] / 256
    res = dict(
        metric="training samples*epochs/s", value=N * steps / wall, unit="samples*epochs/s",
        ms_per_step=wall * 1e3 / steps, dtype="f32",
        config={"workload": f"several hidden layers: N=120 x 33, {'-'.join(map(str, widths))}, full batch, hidden "
                            f"{args.act}, sigmoid output, MSE, GD lr=0.1; every epoch in one launch "
                            "(mlp_deep_train)", "n_rows": N, "widths": widths, "step": "one epoch"},
        graph={"value": N * steps / gwall, "ms_per_step": gwall * 1e3 / steps,
               "form": f"per epoch the dense-layer forward, the squared-error gradient, the dense-layer adjoints and "
                       f"the update as library calls, replayed from a HIP graph of {G} epochs"},
        autograd={"value": N * ag_epochs / awall, "ms_per_step": awall * 1e3 / ag_epochs, "epochs": ag_epochs,
                  "form": "DenseFunction layers composed by torch.autograd, launched from Python"},
        roofline={"bound": "alu", "achieved": achieved, "peak": PEAK["fp32"], "unit": "TFLOP/s",
                  "frac": achieved / PEAK["fp32"], "traffic": None, "traffic_unit": "bytes per launch",
                  "kernel": "mlpk::k_deep_train", "kernel_ms": kern * 1e3, "flops_per_launch": flops,
                  "one_cu": {"peak": cu_peak, "unit": "TFLOP/s", "frac": achieved / cu_peak,
                             "epoch_us": kern * 1e6 / steps}},
        final_loss=final_loss, repeats=reps, steps=steps, warmup=warmup)
    return res, dict(w=w, theta=theta, widths=widths, act=args.act)


def cpu_deep(ctx, budget_s: float):
    import oracle
    w = ctx["w"]
    epochs = 200
    reps, t_total = 0, 0.0
    while (t_total < budget_s or reps == 0) and reps < 100000:
        t0 = time.perf_counter()
        oracle.deep_train(w["X"], w["T"], ctx["widths"], ctx["theta"], 0.1, epochs, act=ctx["act"])
        t_total += time.perf_counter() - t0
        reps += 1
    rows = w["X"].shape[0]
    return {"value": rows * epochs * reps / t_total, "unit": "samples*epochs/s", "cores": 1, "kind": "oracle",
            "sample": f"{rows} rows x {epochs} epochs, run {reps} time(s), float64, single thread, {cpu_info()}",
            "seconds": t_total}


# ---------------------------------------------------------------- differentiation path (w2a)
def bench_autograd(args):
    import torch
    from paper_1908_07847_amd import mlp, synth

    w = synth.single(2)
    D, H, K, N = w["D"], w["H"], w["K"], w["X"].shape[0]
    net = mlp.Net(D, H, K, N, lr=w["lr"], theta=w["theta"])
    X = torch.from_numpy(w["X"]).cuda()
    T = torch.from_numpy(w["T"]).cuda()
    net.flat.requires_grad_(True)
    params = list(mlp.split_packed(net.flat, D, H, K))
    steps = args.steps if args.steps is not None else w["epochs"]
    warmup = args.warmup if args.warmup is not None else 20
    hist = torch.empty(max(steps, warmup, 1), device="cuda")

    def epochs(count):
        for e in range(count):
            Y = mlp.MLPFunction.apply(net, X, *params)
            loss = torch.nn.functional.mse_loss(Y, T)
            gW1, gb1, gW2, gb2 = torch.autograd.grad(loss, params)
            with torch.no_grad():   # the adjoint's own gradient buffers feed the update directly
                net.step(mlp.Grads(gW1, gb1, gW2, gb2, None))
            hist[e] = loss.detach()
    epochs(warmup)
    with torch.no_grad():
        net.set_theta(w["theta"])
    stream = torch.cuda.current_stream()
    wall, kern = timed(lambda: epochs(steps), stream)
    # the same epochs as library calls only (forward, the library's MSE
    # adjoint, update) replayed from a HIP graph of G epochs
    G = 50
    gnet = mlp.Net(D, H, K, N, lr=w["lr"], theta=w["theta"])
    gep = mlp.NetEpochs(gnet, X, T).graph(G)

    def run_graph():
        for r in range(max(steps // G, 1)):
            gep.replay()
    gwall, _ = timed(run_graph, stream)
    gsteps = max(steps // G, 1) * G
    P = D * H + H + H * K + K
    flops = flops_per_sample_epoch(D, H, K) * N * steps + 2 * P * steps
    achieved = flops / kern / 1e12
    res = dict(
        metric="training samples*epochs/s", value=N * steps / wall, unit="samples*epochs/s",
        ms_per_step=wall * 1e3 / steps, dtype="f32",
        config={"workload": "differentiation: N=120 x 33, 33-16-3, full batch, MLPFunction forward + hand-written "
                            "adjoint + mlp_step per epoch (launched from Python)", "n_rows": N, "n_in": D,
                "n_hidden": H, "n_out": K, "lr": w["lr"], "step": "one epoch"},
        roofline={"bound": "alu", "achieved": achieved, "peak": PEAK["fp32"], "unit": "TFLOP/s",
                  "frac": achieved / PEAK["fp32"], "traffic": None, "traffic_unit": "bytes per launch",
                  "kernel": "mlpk::k_forward_tiled + k_backward_rows + k_backward_sum + k_step (per epoch)",
                  "kernel_ms": kern * 1e3, "flops_per_launch": flops},
        graph={"value": N * gsteps / gwall, "ms_per_step": gwall * 1e3 / gsteps, "epochs": gsteps,
               "form": f"per epoch mlp_forward, mlp_backward (the library's MSE adjoint) and mlp_step as library "
                       f"calls, replayed from a HIP graph of {G} epochs (no torch autograd inside the capture)"},
        final_loss=float(hist[steps - 1].item()) if steps else None, steps=steps, warmup=warmup)
    return res, dict(w=w, wl=2, batch=N)


# ---------------------------------------------------------------- predictions (p4)
def bench_predict(args):
    import torch
    from paper_1908_07847_amd import mlp, synth

    w = synth.single(4)
    D, H, K, N = w["D"], w["H"], w["K"], w["X"].shape[0]
    net = mlp.Net(D, H, K, N, batch=w["batch"], theta=w["theta"])
    X = torch.from_numpy(w["X"]).cuda()
    T = torch.from_numpy(w["T"]).cuda()
    steps = args.steps if args.steps is not None else 10
    warmup = args.warmup if args.warmup is not None else 2
    for _ in range(warmup):
        net.predict(X, T)
    stream = torch.cuda.current_stream()

    def run():
        for _ in range(steps):
            net.predict(X, T)
    wall, kern = timed(run, stream)
    reps = repeats(run, stream, wall, steps)
    flops = (2 * D * H + 4 * H + 2 * H * K + 4 * K) * N * steps    # z1, sigma, z2, sigma per row
    achieved = flops / kern / 1e12
    res = dict(
        metric="predicted rows/s", value=N * steps / wall, unit="rows/s", ms_per_step=wall * 1e3 / steps,
        dtype="f32",
        config={"workload": "class predictions of the 33-256-3 net on N=1,048,576 x 33 (forward, argmax, "
                            "correct count)", "n_rows": N, "n_in": D, "n_hidden": H, "n_out": K,
                "step": "one mlp_predict call over all rows"},
        roofline={"bound": "alu", "achieved": achieved, "peak": PEAK["fp32"], "unit": "TFLOP/s",
                  "frac": achieved / PEAK["fp32"], "traffic": measured_traffic(f"p4-fp32-steps{steps}", "layer"),
                  "traffic_unit": "bytes per launch",
                  "kernel": "mlp_predict (mlpk::k_fill_i32 + k_forward_tiled + k_argmax)",
                  "kernel_ms": kern * 1e3 / steps, "flops_per_launch": flops // steps},
        repeats=reps, steps=steps, warmup=warmup)
    return res, dict(w=w)


def cpu_predict(ctx, budget_s: float):
    import oracle
    w = ctx["w"]
    p = oracle.Params.of(w["theta"])
    rows = 65536
    reps, t_total = 0, 0.0
    while (t_total < budget_s or reps == 0) and reps < 100000:
        t0 = time.perf_counter()
        oracle.predict(w["X"][:rows], p)
        t_total += time.perf_counter() - t0
        reps += 1
    return {"value": rows * reps / t_total, "unit": "rows/s", "cores": 1, "kind": "oracle",
            "sample": f"the first {rows} rows, run {reps} time(s), float64, single thread, {cpu_info()}",
            "seconds": t_total}


def copy_probe(n_bytes: int = 1 << 30):
    """A plain device-to-device copy of known size, used to scale the HBM
    byte counters (FETCH_SIZE / WRITE_SIZE) of the profiler."""
    import torch
    a = torch.ones(n_bytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": n_bytes}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default: the workload's epochs)")
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--workload", default="w5", choices=["w1", "w2", "w2a", "w2d", "w3", "w4", "w5", "w6", "p4"])
    ap.add_argument("--prec", default="fp32", choices=["fp32", "bf16", "e4m3"])
    ap.add_argument("--forms", default="all", choices=["all", "none"],
                    help="w4/w5: also time the other operand forms (reported under 'forms' with vs_plain)")
    ap.add_argument("--act", default="sigmoid", choices=["sigmoid", "tanh"],
                    help="hidden activation (w1, w2; tanh is a variant of the paper's sigmoid)")
    ap.add_argument("--momentum", type=float, default=0.0, help="heavy-ball rate (w1, w2; 0 = the paper's GD)")
    ap.add_argument("--cpu-budget", type=float, default=10.0, help="seconds of oracle time for cpu_baseline")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-buckets", action="store_true", help="w3: one launch for all nets (no size groups)")
    ap.add_argument("--copy-probe", action="store_true", help="only run a 1 GiB device copy (counter scale)")
    ap.add_argument("--record-counters", nargs=6, metavar=("KEY", "KIND", "FETCH_CSV", "WRITE_CSV", "COPY_FETCH_CSV",
                                                           "COPY_WRITE_CSV"),
                    help="host only: store the HBM bytes of one launch (one epoch) of the large-N trainer from "
                         "rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE files in profiles/counters.json under KEY, with "
                         "the current source hash of kernel KIND")
    args = ap.parse_args()
    if args.record_counters:
        key, kind, f, w, cf, cw = args.record_counters
        rec = counters_record(f, w, cf, cw, "void mlpk::k_large_train" if kind == "large" else "void mlpk::")
        path = os.path.join(ROOT, "profiles", "counters.json")
        with open(path) as fh:
            allrec = json.load(fh)
        allrec[key] = {"source": kernel_source_hash(kind), "hbm_bytes_per_epoch": rec["hbm_bytes"],
                       "fetch_kib": rec["fetch_kib"], "write_kib": rec["write_kib"],
                       "fetch_scale": rec["fetch_scale"], "write_scale": rec["write_scale"]}
        with open(path, "w") as fh:
            json.dump(allrec, fh, indent=1, sort_keys=True)
        print(json.dumps({key: allrec[key]}))
        return
    if args.copy_probe:
        copy_probe()
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this trainer runs on one GPU; the multi-GPU sharding is designed, not "
                                   "built, so --gpus must be 1"}))
        sys.exit(2)
    if args.workload == "w3":
        res, ctx = bench_batched(args)
        cpu = None if args.no_cpu else cpu_batched(ctx, args.cpu_budget)
    elif args.workload == "w2d":
        res, ctx = bench_deep(args)
        cpu = None if args.no_cpu else cpu_deep(ctx, args.cpu_budget)
    elif args.workload == "w2a":
        res, ctx = bench_autograd(args)
        cpu = None if args.no_cpu else cpu_single(ctx, args.cpu_budget)
    elif args.workload == "p4":
        res, ctx = bench_predict(args)
        cpu = None if args.no_cpu else cpu_predict(ctx, args.cpu_budget)
    elif args.workload == "w6":
        res, ctx = bench_shared(args)
        cpu = None if args.no_cpu else cpu_shared(ctx, args.cpu_budget)
    elif args.workload in ("w4", "w5"):
        res, ctx = bench_large(args)
        cpu = None if args.no_cpu else cpu_large(ctx, args.cpu_budget)
    else:
        res, ctx = bench_single(args)
        cpu = None if args.no_cpu else cpu_single(ctx, args.cpu_budget)
    res.update(n_gpus=1, higher_is_better=True, scaling="weak", vs_baseline=None,
               data="synthetic (seeded generator; the paper's clinical table is not available)")
    res["cpu_baseline"] = cpu
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
