#!/usr/bin/env python3
"""Throughput of the split-step Fourier path on one MI355X.

A step is one ssfm_forward call: every realisation of the batch propagated
through the whole link (all spans and split steps).  The default workload is
the dual-polarisation Manakov link of 10 x 80 km SSMF spans, 100 steps per
span, EDFA 16 dB / NF 5 dB with ASE, 2^16 samples per polarisation, for a
batch of independent realisations (distinct noise keys, 16 distinct symbol
streams tiled over the batch); the field is resident in HBM before timing.

Metric: sample-steps/s = batch * n_samples * (spans * steps_per_span) / time.
One JSON line on stdout.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Manakov SSFM sample-steps/s and fwd+adjoint time at ≤1e-5 rel. field error"
HBM_PEAK_GBS = 8000.0


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--batch", type=int, default=512)
    ap.add_argument("--workload", type=int, default=2, choices=[1, 2, 3, 4, 5],
                    help="2: Manakov 2^16 link over a batch; 4: 256 mixed realisations "
                         "(ssfm_batch against the one-at-a-time loop)")
    ap.add_argument("--single-steps", type=int, default=3,
                    help="timed calls of the batch-1 figure (0 to skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--ldbp-checkpoint-steps", type=int, default=0,
                    help="workload 5: steps between checkpoints (default: the span, "
                         "2 steps); 1 = every step, no recompute in the backward")
    ap.add_argument("--no-autotune", action="store_true",
                    help="use the default launch-shape heuristic instead of measuring")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="minimum CPU time of the oracle baseline sample")
    ap.add_argument("--adjoint", type=int, default=1,
                    help="time one forward+adjoint call on the batch (0 to skip)")
    ap.add_argument("--adjoint-state-gib", type=float, default=-1.0,
                    help="device memory for the adjoint's kept spans (GiB); -1: all "
                         "but 8 GiB of the memory free before the call, 0: none")
    ap.add_argument("--dft16", action="store_true",
                    help="time the radix-16 DFT stage prototype: the FFTs' vector "
                         "butterfly against the matrix-core product (one JSON line)")
    ap.add_argument("--orchestration", action="store_true",
                    help="time the ordering points of a split-step call: a dependent "
                         "kernel boundary (graph replay, direct) against a device-wide "
                         "barrier in one cooperative kernel (one JSON line)")
    ap.add_argument("--launch-events", type=int, default=1,
                    help="time every launch with HIP events for the roofline and the "
                         "kernel breakdowns (0: skip them, e.g. under counter collection)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="first run one device-to-device copy of this many MiB (a "
                         "known-size reference for hardware traffic counters)")
    return ap.parse_args()


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


# translation unit and headers each kernel is compiled from
# steps of learned DBP fused into one forward launch (the library's default)
LDBP_FWD_STEPS = 10

KERNEL_SOURCES = {
    "k3_adj": ("ssfm_adjoint_kernels.hip",),
}
FORWARD_SOURCES = ("ssfm_kernels.hip", "philox_dev.hpp")
SHARED_SOURCES = ("fft_dev.hpp", "kernel_common.hpp", "ssfm_internal.hpp")


def kernel_source_digest(kernel: str) -> str:
    """sha256 over the sources the kernel is built from: a traffic figure
    counts only for the code it was measured on."""
    csrc = os.path.join(ROOT, "paper_2507_03509_amd", "csrc")
    h = hashlib.sha256()
    for name in KERNEL_SOURCES.get(kernel, FORWARD_SOURCES) + SHARED_SOURCES:
        h.update(name.encode())
        h.update(open(os.path.join(csrc, name), "rb").read())
    return h.hexdigest()


def traffic_record(kernel: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it was taken on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    digest = kernel_source_digest(kernel)
    ent = rec.get(kernel)
    if not ent or ent.get("kernel_source_sha256") != digest:
        return None
    return ent


def _oracle_realisation(task):
    """CPU-baseline worker (all-cores leg): one oracle propagation of a
    workload realisation; returns its wall seconds."""
    import numpy as np

    import oracle
    from workloads import CONFIGS, make_field
    wid, r = task
    w = CONFIGS[wid]
    a = make_field(w, seed=w.symbol_seed + r)
    t0 = time.perf_counter()
    oracle.propagate(a, w.link, seed=w.ase_seed, realization=r)
    return time.perf_counter() - t0


def cpu_all_cores(workload: int, budget_s: float):
    """The oracle on every host core (a spawned process per core, one
    realisation each, started before this process touches the GPU): returns
    (realisations, wall seconds, workers)."""
    import concurrent.futures
    import multiprocessing
    workers = max(1, min(16, os.cpu_count() or 1))
    ctx = multiprocessing.get_context("spawn")
    t0 = time.perf_counter()
    with concurrent.futures.ProcessPoolExecutor(max_workers=workers, mp_context=ctx) as ex:
        list(ex.map(_oracle_realisation, [(workload, r) for r in range(workers)]))
    return workers, time.perf_counter() - t0, workers


def bench_dft16(args) -> int:
    """Radix-16 DFT stage: 2^20 transforms of 16 complex FP64 values, 64
    rounds each (values through LDS between rounds, as between FFT passes),
    on the vector butterfly (method 0) and on the FP64 matrix cores
    (method 1).  Flops counted per transform and round: 5 N log2 N = 320 for
    the butterfly (the FFT convention) and 2 x 32 x 32 = 2048 for the matrix
    product (what the matrix cores execute)."""
    import numpy as np
    import torch

    import paper_2507_03509_amd as ssfm

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    ssfm.load_library()
    dev = torch.device("cuda:0")
    count, rounds = 1 << 20, 64
    rng = np.random.default_rng(16)
    x = torch.from_numpy(rng.standard_normal((count, 16)) + 1j * rng.standard_normal((count, 16)))
    data = x.to(dev)
    stream = torch.cuda.current_stream(dev)
    res = {}
    for method, name in ((0, "valu_butterfly"), (1, "mfma_f64_matrix")):
        for _ in range(max(1, args.warmup)):
            ssfm.ssfm_dft16_rounds(method, data, rounds, stream)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            ssfm.ssfm_dft16_rounds(method, data, rounds, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        per_s = count * rounds / (ms * 1e-3)
        flops = 320.0 if method == 0 else 2.0 * 32 * 32
        res[name] = {"ms_per_call": round(ms, 4), "transforms_per_s": per_s,
                     "tflops": per_s * flops / 1e12}
        log(f"{name}: {ms:.3f} ms per call, {per_s:.4e} transforms/s, "
            f"{per_s * flops / 1e12:.1f} TFLOP/s counted")
    out = {
        "metric": "radix-16 DFT stage (FP64) transforms/s", "unit": "transforms/s",
        "value": res["valu_butterfly"]["transforms_per_s"], "higher_is_better": True,
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "dtype": "f64",
        "data": "synthetic", "config": {"workload": "dft16 2^20 transforms x 64 rounds"},
        "methods": res,
        "mfma_over_valu_time": res["valu_butterfly"]["transforms_per_s"] /
                               res["mfma_f64_matrix"]["transforms_per_s"],
    }
    print(json.dumps(out), flush=True)
    return 0


def bench_orchestration(args) -> int:
    """GPU time per ordering point between dependent passes, by workgroup
    count: a boundary between dependent launches of an empty kernel, replayed
    from a graph (method 0) or launched directly (1), against a device-wide
    barrier crossed by every workgroup of one cooperative kernel (2) -- the
    persistent alternative to graph replay for the four-step path, which
    needs two such points per split step."""
    import torch

    import paper_2507_03509_amd as ssfm

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    ssfm.load_library()
    stream = torch.cuda.current_stream(torch.device("cuda:0"))
    rounds = 2000
    res = {}
    for name, method in (("graph_replay", 0), ("direct_launch", 1), ("grid_barrier", 2)):
        res[name] = {}
        for wg in (8, 32, 64, 128, 256, 512):
            ssfm.ssfm_orchestration_probe(method, wg, 100, stream)  # warm-up
            us = min(ssfm.ssfm_orchestration_probe(method, wg, rounds, stream)
                     for _ in range(max(1, args.steps)))
            res[name][str(wg)] = round(us, 3)
            log(f"{name}, {wg} workgroups: {us:.3f} us per ordering point")
    out = {
        "metric": "GPU time per ordering point between dependent passes", "unit": "us",
        "value": res["graph_replay"]["512"], "higher_is_better": False,
        "n_gpus": 1, "steps": args.steps, "warmup": 1, "dtype": "none",
        "data": "synthetic", "config": {"workload": f"{rounds} ordering points, 256-lane workgroups"},
        "us_per_point": res,
    }
    print(json.dumps(out), flush=True)
    return 0


def bench_mixed_batch(args) -> int:
    """Workload 4: 256 independent dual-pol realisations with lengths drawn
    from 2^12..2^16, launch power in [-4, +6] dBm, 1..10 spans of 50 steps and
    distinct seeds -- one ssfm_batch call against one ssfm_forward call per
    realisation."""
    import numpy as np
    import torch

    import paper_2507_03509_amd as ssfm
    from workloads import batch_config, dual_pol_field

    ssfm.load_library()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    items = batch_config(256)
    rng = np.random.default_rng(20250703 + 44)
    links = [it.link() for it in items]
    inputs = [dual_pol_field(rng, 2, ln.n_samples, 2, 64e9, 0.1, it.launch_dbm)
              for it, ln in zip(items, links)]
    seeds = [it.seed for it in items]
    fields = [torch.from_numpy(a.astype(np.complex64)).to(dev) for a in inputs]
    work = sum(ln.n_samples * ln.n_spans * ln.steps_per_span for ln in links)
    stream = torch.cuda.current_stream(dev)
    log(f"workload 4: {len(items)} realisations, {work:.3e} sample-steps per pass")

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    # parity sample: one call on the inputs, then per length group the entry
    # with the most spans against the FP64 oracle
    ssfm.ssfm_batch(links, fields, seeds, 0, stream)
    torch.cuda.synchronize()
    rel_errs = {}
    import oracle
    for n in sorted({ln.n_samples for ln in links}):
        k = max((i for i, ln in enumerate(links) if ln.n_samples == n),
                key=lambda i: links[i].n_spans)
        want = oracle.propagate(inputs[k], links[k], seed=seeds[k], realization=0)
        got = fields[k].cpu().numpy().astype(np.complex128)
        rel_errs[f"entry{k}_n{n}_spans{links[k].n_spans}"] = float(
            np.linalg.norm(got - want) / np.linalg.norm(want))
    log(f"workload 4 parity sample: {rel_errs}")
    for f, a in zip(fields, inputs):
        f.copy_(torch.from_numpy(a.astype(np.complex64)))
    torch.cuda.synchronize()
    # every call launched directly (SSFM_GRAPH=0), then the library's default:
    # a repeated call replays the captured launch sequence (the warm-up call
    # of `timed` captures it, after measuring the groups' launch shapes)
    os.environ["SSFM_GRAPH"] = "0"
    ms_direct = timed(lambda: ssfm.ssfm_batch(links, fields, seeds, 0, stream), args.steps)
    del os.environ["SSFM_GRAPH"]
    ms_batch = timed(lambda: ssfm.ssfm_batch(links, fields, seeds, 0, stream), args.steps)
    plans = {}
    for ln in links:
        key = (ln.n_samples,)
        if key not in plans:
            plans[key] = ssfm.Plan(ln.replace(n_spans=10), device=0)

    def loop():
        for ln, f, sd in zip(links, fields, seeds):
            plans[(ln.n_samples,)].forward(f, seed=sd, span_end=ln.n_spans, stream=stream)

    ms_loop = timed(loop, max(1, args.steps // 2))
    value = work / (ms_batch / 1e3)
    loop_rate = work / (ms_loop / 1e3)
    log(f"ssfm_batch direct launches: {ms_direct:.2f} ms per pass")
    log(f"ssfm_batch: {ms_batch:.2f} ms per pass ({value:.4e} sample-steps/s); "
        f"one-at-a-time: {ms_loop:.2f} ms ({loop_rate:.4e}); speedup {ms_loop / ms_batch:.2f}x")
    out = {
        "metric": METRIC, "value": value, "unit": "sample-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": 1, "ms_per_step": round(ms_batch, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "mixed batch: 256 dual-pol realisations, 2^12..2^16 samples, "
                               "1..10 x 80 km spans of 50 steps, -4..+6 dBm, distinct seeds",
                   "sample_steps_per_pass": work, "parallelism": "single-gpu"},
        "one_at_a_time": {"ms_per_pass": round(ms_loop, 3), "sample_steps_per_s": loop_rate},
        "batch_direct_launches": {"ms_per_pass": round(ms_direct, 3),
                                  "note": "ssfm_batch with graph replay off (SSFM_GRAPH=0)"},
        "batched_speedup": round(ms_loop / ms_batch, 3),
        "rel_err_vs_oracle": max(rel_errs.values()), "rel_err_sampled": rel_errs,
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)
    for pl in plans.values():
        pl.close()
    return 0


def bench_ldbp(args) -> int:
    """Workload 5: learned digital back-propagation over 64 received dual-pol
    fields of 2^14 samples (10 x 80 km, 2 steps per span, 15 taps).  A
    training step is forward with span checkpoints, matched-filter MSE with
    its gradient, and the backward pass; its time is compared with the
    forward-and-loss time (fwd+adjoint / fwd)."""
    import numpy as np
    import torch

    import paper_2507_03509_amd as ssfm
    from paper_2507_03509_amd import ldbp
    from workloads import LDBP, field_and_targets, rrc_taps

    ssfm.load_library()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    cfg = LDBP
    w = cfg.workload
    ln = w.link
    B, P, N, K = cfg.batch, ln.n_pol, ln.n_samples, cfg.n_steps
    mf = rrc_taps(w.sps, w.rolloff, cfg.mf_half)
    rng = np.random.default_rng(w.symbol_seed)
    tx, tg = [], []
    for _ in range(B):
        f, t = field_and_targets(rng, P, N, w.sps, w.symbol_rate_hz, w.rolloff, w.launch_dbm, mf)
        tx.append(f)
        tg.append(t)
    # received fields: this library's own propagation over the link (untimed)
    x = torch.from_numpy(np.stack(tx).astype(np.complex64)).to(dev)
    plan = ssfm.Plan(ln, device=0)
    plan.forward(x, seed=w.ase_seed)
    sym = torch.from_numpy(np.stack(tg).astype(np.complex64)).to(dev)
    mfd = torch.from_numpy(mf).to(dev)
    taps_h, xi_h = ldbp.init_params(ln, cfg.n_taps, cfg.steps_per_span)
    taps = torch.from_numpy(taps_h).to(dev)
    xi = torch.from_numpy(xi_h).to(dev)
    ck_steps = args.ldbp_checkpoint_steps or cfg.steps_per_span
    model = ldbp.Ldbp(n_pol=P, n_steps=K, n_taps=cfg.n_taps, steps_per_span=ck_steps,
                      n_samples=N, sps=w.sps, mf_taps=2 * cfg.mf_half + 1, device=0)
    ck = model.new_checkpoints(B)
    stream = torch.cuda.current_stream(dev)
    state = {}

    def fwd():
        z = model.forward(x, taps, xi)
        state["loss"], _ = model.loss(z, sym, mfd, want_grad=False)

    def train():
        z = model.forward(x, taps, xi, ck)
        loss, g = model.loss(z, sym, mfd, want_grad=True)
        state["grads"] = model.backward(x, z, taps, xi, ck, g)
        state["loss"] = loss

    def timed(fn, reps):
        for _ in range(max(1, args.warmup)):
            fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    reps = max(10, 10 * args.steps)
    ms_fwd = timed(fwd, reps)
    ms_train = timed(train, reps)
    # the forward kernel alone, for the roofline: the library fuses up to
    # LDBP_FWD_STEPS steps per launch, so a call is ceil(K / that) equal launches
    ms_fwd_kernel = timed(lambda: model.forward(x, taps, xi), reps)
    fwd_launches = -(-K // LDBP_FWD_STEPS)
    # the backward call alone (its cotangent, overwritten by each call, is
    # restored from a copy first: one 2 x 2^14 x 64 complex64 copy per call)
    zb = model.forward(x, taps, xi, ck)
    _, gb = model.loss(zb, sym, mfd, want_grad=True)
    gw = gb.clone()

    def bwd():
        gw.copy_(gb)
        model.backward(x, zb, taps, xi, ck, gw)

    ms_bwd = timed(bwd, reps)
    # algorithmic FP64 flops of the backward per span and sample: the span's
    # inner states recomputed (S - 1 forward steps) and S reverse steps of FIR
    # transpose (8 T P), tap gradient (8 T P) and Kerr pullback (~25 P)
    S = cfg.steps_per_span
    fwd_step_flops = P * 8 * cfg.n_taps + 9 * P + 1
    rev_step_flops = 2 * P * 8 * cfg.n_taps + 25 * P
    bwd_flops = B * N * (K // S) * ((S - 1) * fwd_step_flops + S * rev_step_flops)
    bwd_tflops = bwd_flops / (ms_bwd * 1e-3) / 1e12
    work = B * N * K                                   # sample-steps per pass
    # algorithmic FP64 flops per sample-step: FIR 8 T per polarisation
    # (T complex multiply-adds), Kerr 3 P (|y|^2) + 1 (phase) + 6 P (rotation);
    # the phasor itself is not counted
    flops = P * 8 * cfg.n_taps + 9 * P + 1
    achieved = work * flops / (ms_fwd_kernel * 1e-3) / 1e12
    peak = 78.6
    value = work / (ms_train / 1e3)
    log(f"LDBP {B} x {P} x 2^{int(math.log2(N))}, K={K}: forward+loss {ms_fwd:.3f} ms, "
        f"train step {ms_train:.3f} ms ({ms_train / ms_fwd:.2f}x), forward kernel "
        f"{ms_fwd_kernel:.3f} ms = {achieved:.1f} TFLOP/s FP64, backward call {ms_bwd:.3f} ms = "
        f"{bwd_tflops:.1f} TFLOP/s FP64, loss {float(state['loss'][0]):.4e}")
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        x_h = x[:1].cpu().numpy().astype(np.complex128)
        s_h = sym[:1].cpu().numpy().astype(np.complex128)
        t0 = time.perf_counter()
        done = 0
        while True:
            zo = oracle.ldbp_forward(x_h, taps_h, xi_h)
            gzo = oracle.mse_grad(zo, s_h, mf, w.sps) / B   # loss normalised over the batch
            oracle.ldbp_backward(x_h, taps_h, xi_h, gzo)
            done += 1
            if time.perf_counter() - t0 >= min(args.cpu_seconds, 30.0):
                break
        csec = time.perf_counter() - t0
        cpu = {"value": done * N * K / csec, "unit": "sample-steps/s", "cores": 1,
               "kind": "oracle",
               "sample": f"{done} realisation(s) of 1 x {P} x {N}: forward, loss gradient "
                         f"and backward in {csec:.1f} s"}
        log(f"oracle training step: {done} realisation(s) in {csec:.1f} s")
    out = {
        "metric": "LDBP training step sample-steps/s (forward, MSE, backward) at <=1e-5 rel. error",
        "value": value, "unit": "sample-steps/s", "n_gpus": 1, "steps": reps,
        "warmup": max(1, args.warmup), "ms_per_step": round(ms_train, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"learned DBP: {B} x {P}-pol x {N} received fields, "
                               f"{ln.n_spans} x {ln.span_km:g} km, {cfg.steps_per_span} "
                               f"steps/span, {cfg.n_taps} taps, MSE through a "
                               f"{2 * cfg.mf_half + 1}-tap RRC matched filter",
                   "checkpoint_every_steps": ck_steps,
                   "sample_steps_per_pass": work, "parallelism": "single-gpu"},
        "ms_forward_and_loss": round(ms_fwd, 4), "ms_train_step": round(ms_train, 4),
        "fwd_adjoint_over_fwd": round(ms_train / ms_fwd, 3),
        "backward": {"ms_per_call": round(ms_bwd, 4), "achieved_tflops": round(bwd_tflops, 2),
                     "frac": round(bwd_tflops / 78.6, 4),
                     "algorithmic_flops_per_call": bwd_flops,
                     "note": "includes one cotangent copy per call"},
        "roofline": {"bound": "alu", "achieved": round(achieved, 2), "peak": peak,
                     "unit": "TFLOP/s", "frac": round(achieved / peak, 4), "traffic": None,
                     "kernel": "ldbp_fwd",
                     "avg_launch_us": round(ms_fwd_kernel * 1e3 / fwd_launches, 2),
                     "algorithmic_flops_per_launch": work * flops // fwd_launches,
                     "launches_per_forward": fwd_launches},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    model.close()
    plan.close()
    return 0


def main() -> int:
    args = parse()
    if args.dft16 and args.gpus == 1:
        return bench_dft16(args)
    if args.orchestration and args.gpus == 1:
        return bench_orchestration(args)
    if args.workload == 4 and args.gpus == 1:
        return bench_mixed_batch(args)
    if args.workload == 5 and args.gpus == 1:
        return bench_ldbp(args)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the SSFM "
              "path has no multi-GPU code", file=sys.stderr)
        return 2

    # all-cores oracle leg first: its worker processes are spawned before this
    # process initialises the GPU
    cpu_all = None
    if not args.no_cpu_baseline:
        done_all, sec_all, workers = cpu_all_cores(args.workload, args.cpu_seconds)
        cpu_all = (done_all, sec_all, workers)
        log(f"oracle on {workers} cores: {done_all} realisation(s) in {sec_all:.1f} s")

    import numpy as np
    import torch

    import paper_2507_03509_amd as ssfm
    from workloads import CONFIGS, make_field

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    ssfm.load_library()  # raises if the HIP library is not built
    w = CONFIGS[args.workload]
    link = w.link
    n, p = link.n_samples, link.n_pol
    total_steps = link.n_spans * link.steps_per_span
    batch = args.batch
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    if args.copy_calibration_mib > 0:
        nbytes = args.copy_calibration_mib << 20
        src = torch.empty(nbytes // 4, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: {nbytes} bytes read + {nbytes} bytes written")
        del src, dst

    # ---- inputs: resident in HBM before timing -------------------------------
    distinct = min(batch, 16)
    host = np.stack([make_field(w, seed=w.symbol_seed + i) for i in range(distinct)])
    base = torch.from_numpy(host.astype(np.complex64)).to(dev)
    reps = (batch + distinct - 1) // distinct
    field = base.repeat(reps, 1, 1)[:batch].contiguous()
    ref_in = host[0].copy()
    plan = ssfm.Plan(link, device=0)
    info = plan.info
    stream = torch.cuda.current_stream(dev)
    log(f"workload {w.name} batch={batch} plan={info}")
    # launch shapes by measurement for every batch size timed below (untimed;
    # the shapes do not change results)
    tuned = {}
    if not args.no_autotune:
        for bsz in sorted({batch, 64, 1}):
            if bsz <= batch:
                tuned[bsz] = plan.autotune(bsz, stream)
                log(f"autotune batch {bsz}: columns {tuned[bsz]['columns']}, row workgroup "
                    f"{tuned[bsz]['row_lanes']} lanes, us/step {tuned[bsz]['us_per_step']}")

    # ---- first call doubles as the parity sample (realisation 0) ------------
    plan.forward(field, seed=w.ase_seed, stream=stream)
    torch.cuda.synchronize()
    gpu_out0 = field[0].cpu().numpy().astype(np.complex128)
    for _ in range(max(0, args.warmup - 1)):
        plan.forward(field, seed=w.ase_seed, stream=stream)
    torch.cuda.synchronize()

    # the library's default (documented with ssfm_plan_set_forward_streams):
    # each chunk as two concurrent parts when each part holds >= 256 column
    # tiles
    sub_batches = 1
    if info["path"] == 2:
        chunk = info["chunk_realisations"] or batch
        chunk = -(-batch // -(-batch // chunk))
        sub_batches = 2 if chunk * info["n2"] // info["columns_per_tile"] >= 512 else 1
    # ---- timed region: K calls as the library runs them ---------------------
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    wall0 = time.perf_counter()
    t0.record(stream)
    for _ in range(args.steps):
        plan.forward(field, seed=w.ase_seed, stream=stream)
    t1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms_total = t0.elapsed_time(t1)
    ms_per_step = ms_total / args.steps
    value = batch * n * total_steps / (ms_per_step / 1e3)
    log(f"timed {args.steps} calls: {ms_per_step:.3f} ms/call, wall {wall:.3f}s, "
        f"{value:.4e} sample-steps/s")

    if args.launch_events:
        # ---- kernel rates: K single-stream calls with HIP events around every
        # launch on the launch stream (the events also turn graph replay off) ----
        plan.set_forward_streams(1)
        ssfm.ssfm_profile_begin(plan.handle)
        torch.cuda.synchronize()
        k0 = torch.cuda.Event(enable_timing=True)
        k1 = torch.cuda.Event(enable_timing=True)
        k0.record(stream)
        for _ in range(args.steps):
            plan.forward(field, seed=w.ase_seed, stream=stream)
        k1.record(stream)
        torch.cuda.synchronize()
        stats = ssfm.ssfm_profile_end(plan.handle)
        plan.set_forward_streams(0)
        ms_single = k0.elapsed_time(k1) / args.steps
        log(f"single-stream calls with per-launch events: {ms_single:.3f} ms/call")
        for s in stats:
            log(f"  {s['name']}: {s['launches']} launches, {s['total_ms']:.3f} ms, "
                f"{s['field_bytes'] / (s['total_ms'] * 1e-3) / 1e9:.1f} GB/s algorithmic")

        dom = max(stats, key=lambda s: s["total_ms"])
        per_launch_ms = dom["total_ms"] / dom["launches"]
        bytes_per_launch = dom["field_bytes"] / dom["launches"]
        achieved = bytes_per_launch / (per_launch_ms * 1e-3) / 1e9
        tr = traffic_record(dom["name"])
        roofline = {
            "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": tr["bytes_per_launch"] if tr else None,
            "kernel": dom["name"], "avg_launch_us": round(per_launch_ms * 1e3, 3),
            "measured_on": "single-stream calls of the full batch (run by the library as "
                           "cache-sized chunks), HIP events around every launch",
            "single_stream_ms_per_call": round(ms_single, 3),
            "path_gbs": round(2 * 2 * batch * p * n * 8 * total_steps / (ms_per_step * 1e-3) / 1e9, 1),
            "algorithmic_bytes_per_launch": bytes_per_launch,
            "kernels": {s["name"]: {"launches": s["launches"],
                                    "avg_us": round(s["total_ms"] / s["launches"] * 1e3, 3),
                                    "gbs": round(s["field_bytes"] / (s["total_ms"] * 1e-3) / 1e9, 1)}
                        for s in stats},
        }
    else:
        roofline = None

    # ---- forward + adjoint (one ssfm_adjoint call: forward with span
    # checkpoints, then the reverse sweep) on the same batch -----------------
    adj = None
    if args.adjoint:
        grad = field.clone()

        def time_adjoint(label, reps=3):
            plan.adjoint(field, grad, seed=w.ase_seed, stream=stream)  # workspace + warm-up
            torch.cuda.synchronize()
            times = []
            for _ in range(reps):
                a0 = torch.cuda.Event(enable_timing=True)
                a1 = torch.cuda.Event(enable_timing=True)
                a0.record(stream)
                plan.adjoint(field, grad, seed=w.ase_seed, stream=stream)
                a1.record(stream)
                torch.cuda.synchronize()
                times.append(a0.elapsed_time(a1))
            ms = sorted(times)[len(times) // 2]  # median
            # per-kernel breakdown of one more call (events around every
            # launch; one stream, so that no two launches' windows overlap)
            if args.launch_events:
                plan.set_forward_streams(1)
                ssfm.ssfm_profile_begin(plan.handle)
                plan.adjoint(field, grad, seed=w.ase_seed, stream=stream)
                torch.cuda.synchronize()
                plan.set_forward_streams(0)
                for s_ in ssfm.ssfm_profile_end(plan.handle):
                    log(f"  adjoint call ({label}) {s_['name']}: {s_['launches']} launches, "
                        f"{s_['total_ms']:.1f} ms, "
                        f"{s_['field_bytes'] / (s_['total_ms'] * 1e-3) / 1e9:.1f} GB/s "
                        "algorithmic")
            log(f"forward+adjoint ({label}): median {ms:.3f} ms of {reps} "
                f"({', '.join(f'{t:.1f}' for t in times)}), {ms / ms_per_step:.2f}x forward")
            return ms, times

        # the adjoint runs the batch in sequential chunks of two-field working
        # sets (half the plan's forward chunk), its workspace sized for one
        c2 = plan.info["chunk_realisations"] // 2
        cb = batch
        if 0 < c2 < batch:
            parts = -(-batch // c2)
            cb = -(-batch // parts)
        # the headline: span checkpoints, every span's states rebuilt inside
        # the reverse sweep (no stored states)
        plan.set_state_memory(0)
        ms_rebuild, t_rebuild = time_adjoint("span checkpoints, in-span rebuild")
        adj = {"scheme": "span checkpoints + in-span recomputation (no stored states)",
               "fwd_adjoint_ms": round(ms_rebuild, 3),
               "ratio_to_forward": round(ms_rebuild / ms_per_step, 3),
               "timed_calls_ms": [round(t, 3) for t in t_rebuild],
               # span checkpoints of the whole batch (the forward pass runs
               # over all chunks first) and a two-chunk work buffer
               "workspace_gib": round((link.n_spans * batch + 2 * cb) * p * n * 8 / 2 ** 30, 2),
               "realisations_per_chunk": cb,
               "kept_state": None}
        # trailing spans kept: their nonlinear-step inputs stored by the forward
        if args.adjoint_state_gib != 0:
            span_bytes = link.steps_per_span * cb * link.n_pol * link.n_samples * 8
            if args.adjoint_state_gib > 0:
                budget = int(args.adjoint_state_gib * 2 ** 30)
            else:
                budget = max(0, torch.cuda.mem_get_info()[0] - 8 * 2 ** 30)
            kept = min(link.n_spans, budget // span_bytes)
            if kept > 0:
                plan.set_state_memory(kept * span_bytes)
                ms_kept, t_kept = time_adjoint(f"{kept} of {link.n_spans} spans kept per chunk "
                                               f"of {cb}")
                plan.set_state_memory(0)
                # a different scheme (memory for work), reported beside the
                # headline, never in its place
                adj["kept_state"] = {
                    "scheme": "nonlinear-step inputs of the last spans stored by the forward",
                    "fwd_adjoint_ms": round(ms_kept, 3),
                    "ratio_to_forward": round(ms_kept / ms_per_step, 3),
                    "timed_calls_ms": [round(t, 3) for t in t_kept],
                    "kept_spans": int(kept),
                    "realisations_per_chunk": cb,
                    "state_gib": round(kept * span_bytes / 2 ** 30, 1)}
        del grad

    # ---- one field (batch 1): the latency-bound figure ----------------------
    single = None
    if args.single_steps > 0 and batch > 1:
        f1 = field[:1].clone()
        # two untimed calls: the second identical call captures the launch
        # sequence that the timed calls replay
        plan.forward(f1, seed=w.ase_seed, stream=stream)
        plan.forward(f1, seed=w.ase_seed, stream=stream)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.single_steps):
            plan.forward(f1, seed=w.ase_seed, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ms1 = e0.elapsed_time(e1) / args.single_steps
        single = {"ms_per_call": round(ms1, 3),
                  "us_per_split_step": round(ms1 * 1e3 / total_steps, 3),
                  "sample_steps_per_s": n * total_steps / (ms1 / 1e3)}
        log(f"batch 1: {ms1:.3f} ms/call, {single['sample_steps_per_s']:.4e} sample-steps/s")

    # ---- batch 64: 64 MiB of field, resident in the 256 MB last-level cache --
    b64 = None
    if args.single_steps > 0 and batch >= 64:
        f64 = field[:64].clone()
        plan.forward(f64, seed=w.ase_seed, stream=stream)
        plan.forward(f64, seed=w.ase_seed, stream=stream)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.single_steps):
            plan.forward(f64, seed=w.ase_seed, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ms64 = e0.elapsed_time(e1) / args.single_steps
        b64 = {"ms_per_call": round(ms64, 3),
               "us_per_split_step": round(ms64 * 1e3 / total_steps, 3),
               "sample_steps_per_s": 64 * n * total_steps / (ms64 / 1e3)}
        log(f"batch 64: {ms64:.3f} ms/call, {b64['sample_steps_per_s']:.4e} sample-steps/s")
        # forward+adjoint at this batch with the nonlinear-step inputs of as
        # many spans kept as the free memory holds (every span, normally)
        if args.adjoint and args.adjoint_state_gib != 0:
            span64 = link.steps_per_span * 64 * link.n_pol * link.n_samples * 8
            free = max(0, torch.cuda.mem_get_info()[0] - 8 * 2 ** 30)
            kept64 = min(link.n_spans, free // span64)
            if kept64 > 0:
                g64 = f64.clone()
                plan.set_state_memory(kept64 * span64)
                plan.adjoint(f64, g64, seed=w.ase_seed, stream=stream)  # store + warm-up
                torch.cuda.synchronize()
                t64 = []
                for _ in range(3):
                    e0.record(stream)
                    plan.adjoint(f64, g64, seed=w.ase_seed, stream=stream)
                    e1.record(stream)
                    torch.cuda.synchronize()
                    t64.append(e0.elapsed_time(e1))
                ms64a = sorted(t64)[1]
                plan.set_state_memory(0)
                b64.update({"kept_state_fwd_adjoint_ms": round(ms64a, 3),
                            "kept_state_fwd_adjoint_ratio": round(ms64a / ms64, 3),
                            "kept_spans": int(kept64),
                            "state_gib": round(kept64 * span64 / 2 ** 30, 1)})
                log(f"batch 64 forward+adjoint, {kept64} of {link.n_spans} spans kept: "
                    f"{ms64a:.3f} ms ({ms64a / ms64:.2f}x forward)")
                del g64
        del f64

    # ---- achievable bandwidth: this library's plain copy kernel on the
    # batch field (read + write of 2^29 bytes) -------------------------------
    dst = torch.empty_like(field)
    ssfm.ssfm_stream_copy(dst, field, stream)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(5):
        ssfm.ssfm_stream_copy(dst, field, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    copy_gbs = 2 * field.numel() * 8 / (e0.elapsed_time(e1) / 5 * 1e-3) / 1e9
    if roofline is not None:
        roofline["copy_kernel_gbs"] = round(copy_gbs, 1)
        roofline["frac_of_copy"] = round(achieved / copy_gbs, 4)
        log(f"copy kernel: {copy_gbs:.1f} GB/s (the column pass reaches "
            f"{achieved / copy_gbs:.2f} of it)")
    del dst

    # ---- CPU oracle on one realisation (also the parity reference) ----------
    cpu = None
    rel_err = None
    if not args.no_cpu_baseline:
        # realisation 0 doubles as the parity reference; further realisations
        # (their own inputs and noise keys) until ~10 s of CPU work
        import oracle
        c0 = time.perf_counter()
        want = oracle.propagate(ref_in, link, seed=w.ase_seed, realization=0)
        done = 1
        rel_err = float(np.linalg.norm(gpu_out0 - want) / np.linalg.norm(want))
        while time.perf_counter() - c0 < args.cpu_seconds and done < min(distinct, 8):
            oracle.propagate(host[done], link, seed=w.ase_seed, realization=done)
            done += 1
        csec = time.perf_counter() - c0
        cpu = {"value": done * n * total_steps / csec, "unit": "sample-steps/s", "cores": 1,
               "kind": "oracle",
               "sample": f"{done} realisation(s) of the same link ({link.n_spans} spans x "
                         f"{link.steps_per_span} steps, {n} samples x {p} pol), FP64 NumPy, "
                         f"{csec:.1f} s on {cpu_model()} ({os.cpu_count()} logical CPUs, "
                         "single-threaded FFT and elementwise ops)"}
        log(f"oracle: {done} realisation(s) in {csec:.1f} s; rel err of GPU realisation 0 = "
            f"{rel_err:.3e}")

    out = {
        "metric": METRIC, "value": value, "unit": "sample-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{w.name} x{batch} realisations",
                   "n_samples": n, "n_pol": p, "spans": link.n_spans,
                   "steps_per_span": link.steps_per_span, "batch": batch,
                   "field_storage": "complex64", "linear_step_arithmetic": "f64",
                   "parallelism": "single-gpu",
                   "concurrent_sub_batches": sub_batches},
        "rel_err_vs_oracle": rel_err,
        "fwd_adjoint_ms": adj["fwd_adjoint_ms"] if adj else None,
        "fwd_adjoint_ratio": adj["ratio_to_forward"] if adj else None,
        "fwd_adjoint": adj,
        "pol_sample_steps_per_s": value * p,
        "batch1": single,
        "batch64": b64,
        "launch_shapes": {str(k): {"columns": v["columns"], "row_lanes": v["row_lanes"]}
                          for k, v in tuned.items()},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "cpu_baseline_all_cores": None if cpu_all is None else {
            "value": cpu_all[0] * n * total_steps / cpu_all[1], "unit": "sample-steps/s",
            "cores": cpu_all[2], "kind": "oracle",
            "sample": f"{cpu_all[0]} realisation(s), one per spawned process, in "
                      f"{cpu_all[1]:.1f} s wall"},
    }
    print(json.dumps(out), flush=True)
    plan.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
