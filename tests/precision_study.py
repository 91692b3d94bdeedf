#!/usr/bin/env python3
"""Precision study of the split-step path: relative L2 field error against
the FP64 oracle versus the number of split steps, and per workload.

Compared with the oracle (plain FP64 NumPy, the reference):
  * gpu-fp64  -- the library's path (FP64 registers, complex64 field store);
  * gpu-fp32  -- the library's FP32-arithmetic variant
                 (SSFM_FLAG_FP32_ARITHMETIC: FP32 butterflies, twiddles and
                 nonlinear rotation, FP64 dispersion multiply);
  * cpu-c64   -- a CPU control: the same scheme in complex64 with NumPy's
                 single-precision FFT (pocketfft) and the dispersion factor
                 rounded to complex64.

Part 1 sweeps the step count of workload 2's link (10 x 80 km, 2^16 samples
per polarisation, dual polarisation, EDFA + ASE) from 100 to 4000 split steps
(10..400 steps per span).  Part 2 takes workloads 1-3 at their stated step
counts.  Every input is the seeded synthetic field of the workload.

Run on a host with the GPU (CPU work runs first, in worker processes):

    python tests/precision_study.py --out gpurun_out/precision.json

It prints one markdown table per part.  ``--quick`` shrinks part 1 to 2^14
samples and drops workload 3 (a few seconds of CPU).
"""

from __future__ import annotations

import argparse
import concurrent.futures as cf
import json
import math
import multiprocessing as mp
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

STEPS_PER_SPAN = (10, 20, 50, 100, 200, 400)


def rel(a, b) -> float:
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def propagate_c64(field, link, seed: int, span_begin: int = 0, span_end=None) -> np.ndarray:
    """The oracle's scheme in complex64: NumPy's single-precision FFT, the
    linear factor and the nonlinear rotation rounded to complex64, the noise
    of the oracle rounded to complex64 (a control for the FP32 floor)."""
    import oracle
    p = oracle.si_params(link)
    a = np.array(field, dtype=np.complex64)
    omega = oracle.angular_frequency(p["n"], p["fs"])
    h = p["h"]
    half = oracle.linear_factor(p["beta2"], p["alpha"], omega, h / 2.0).astype(np.complex64)
    full = oracle.linear_factor(p["beta2"], p["alpha"], omega, h).astype(np.complex64)
    coef = np.float32(p["c_nl"] * p["gamma"] * oracle.nl_step_length(p["alpha"], h))
    gain = np.float32(math.sqrt(p["gain"]))
    amplified = p["gain"] != 1.0 or p["ase"]

    def lin(x, f):
        return np.fft.ifft(f * np.fft.fft(x, axis=-1), axis=-1).astype(np.complex64)

    for s in range(span_begin, p["n_spans"] if span_end is None else span_end):
        a = lin(a, half)
        for j in range(p["steps"]):
            power = np.sum(a.real * a.real + a.imag * a.imag, axis=0, keepdims=True)
            ph = coef * power
            a = a * (np.cos(ph) + 1j * np.sin(ph)).astype(np.complex64)
            a = lin(a, full if j < p["steps"] - 1 else half)
        if amplified:
            a = a * gain
            if p["ase"] and p["gain"] > 1.0:
                a = a + oracle.ase_noise(p, seed, 0, s).astype(np.complex64)
    return a


def _cpu_case(args):
    kind, workload, steps, n_samples = args
    import oracle
    from workloads import CONFIGS, make_field
    w = CONFIGS[workload]
    link = w.link if steps is None else w.link.replace(steps_per_span=steps)
    if n_samples is not None:
        link = link.replace(n_samples=n_samples)
    field = make_field(w, seed=w.symbol_seed) if n_samples is None else \
        _small_field(w, n_samples)
    t0 = time.perf_counter()
    out = field
    # span by span (the same arithmetic as one call), reporting progress on
    # the long runs
    for sp in range(link.n_spans):
        if kind == "oracle":
            out = oracle.propagate(out, link, seed=w.ase_seed, span_begin=sp, span_end=sp + 1)
        else:
            out = propagate_c64(out, link, w.ase_seed, span_begin=sp, span_end=sp + 1)
        if time.perf_counter() - t0 > 30 and sp + 1 < link.n_spans:
            print(f"  {kind} workload {workload} steps/span {steps}: span {sp + 1} of "
                  f"{link.n_spans} done", flush=True)
    return (kind, workload, steps, n_samples), out, time.perf_counter() - t0


def _small_field(w, n):
    from workloads import dual_pol_field
    rng = np.random.default_rng(w.symbol_seed)
    return dual_pol_field(rng, w.link.n_pol, n, 2, 64e9, 0.1, 2.0)


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--out", default=None)
    ap.add_argument("--quick", action="store_true")
    ap.add_argument("--workers", type=int, default=min(16, os.cpu_count() or 1))
    args = ap.parse_args()

    sweep_n = (1 << 14) if args.quick else None
    workloads = (1, 2) if args.quick else (1, 2, 3)
    jobs = []
    for k in STEPS_PER_SPAN:
        for kind in ("oracle", "c64"):
            jobs.append((kind, 2, k, sweep_n))
    for wl in workloads:
        for kind in ("oracle", "c64"):
            jobs.append((kind, wl, None, None))
    # CPU work first, before this process touches the GPU
    cpu = {}
    ctx = mp.get_context("spawn")
    with cf.ProcessPoolExecutor(max_workers=args.workers, mp_context=ctx) as ex:
        futs = [ex.submit(_cpu_case, j) for j in jobs]
        for fut in cf.as_completed(futs):
            key, out, sec = fut.result()
            cpu[key] = out
            print(f"cpu {key[0]:6s} workload {key[1]} steps/span {key[2]} n {key[3]}: "
                  f"{sec:.1f} s", flush=True)

    import torch
    import paper_2507_03509_amd as ssfm
    from workloads import CONFIGS, make_field
    assert torch.cuda.is_available(), "the precision study needs the GPU"
    ssfm.load_library()

    def gpu(workload, steps, n_samples, arithmetic):
        w = CONFIGS[workload]
        link = w.link if steps is None else w.link.replace(steps_per_span=steps)
        if n_samples is not None:
            link = link.replace(n_samples=n_samples)
        field = make_field(w, seed=w.symbol_seed) if n_samples is None else \
            _small_field(w, n_samples)
        t = torch.from_numpy(np.asarray(field).astype(np.complex64))[None].cuda()
        plan = ssfm.Plan(link, arithmetic=arithmetic)
        try:
            plan.forward(t, seed=w.ase_seed)
            torch.cuda.synchronize()
        finally:
            plan.close()
        return t[0].cpu().numpy().astype(np.complex128)

    rows1 = []
    for k in STEPS_PER_SPAN:
        ref = cpu[("oracle", 2, k, sweep_n)]
        row = dict(steps=10 * k,
                   cpu_c64=rel(cpu[("c64", 2, k, sweep_n)].astype(np.complex128), ref),
                   gpu_fp64=rel(gpu(2, k, sweep_n, "fp64"), ref),
                   gpu_fp32=rel(gpu(2, k, sweep_n, "fp32"), ref))
        rows1.append(row)
        print(f"sweep {row}", flush=True)
    rows2 = []
    for wl in workloads:
        ref = cpu[("oracle", wl, None, None)]
        w = CONFIGS[wl]
        row = dict(workload=wl, name=w.name, steps=w.link.n_spans * w.link.steps_per_span,
                   cpu_c64=rel(cpu[("c64", wl, None, None)].astype(np.complex128), ref),
                   gpu_fp64=rel(gpu(wl, None, None, "fp64"), ref),
                   gpu_fp32=rel(gpu(wl, None, None, "fp32"), ref))
        rows2.append(row)
        print(f"workload {row}", flush=True)

    n_sweep = sweep_n or CONFIGS[2].link.n_samples
    print(f"\nPart 1: workload 2 link (10 x 80 km, dual pol, 2^{int(math.log2(n_sweep))} "
          "samples/pol), rel. L2 error vs the FP64 oracle")
    print("| split steps | GPU FP64 (library) | GPU FP32 arithmetic | CPU complex64 control |")
    print("|---|---|---|---|")
    for r in rows1:
        print(f"| {r['steps']} | {r['gpu_fp64']:.2e} | {r['gpu_fp32']:.2e} | {r['cpu_c64']:.2e} |")
    print("\nPart 2: workloads at their stated step counts")
    print("| workload | split steps | GPU FP64 (library) | GPU FP32 arithmetic | CPU complex64 control |")
    print("|---|---|---|---|---|")
    for r in rows2:
        print(f"| {r['workload']} {r['name']} | {r['steps']} | {r['gpu_fp64']:.2e} | "
              f"{r['gpu_fp32']:.2e} | {r['cpu_c64']:.2e} |")
    if args.out:
        os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
        with open(args.out, "w") as f:
            json.dump(dict(sweep=rows1, workloads=rows2, sweep_n=n_sweep), f, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
