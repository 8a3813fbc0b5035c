"""Benchmark of the light-curve generator on one MI355X.

A step is one agn_lc_generate_batch call over the whole workload: Timmer-
Koenig moduli for every curve, the one-time sort of every PDF draw, and all
iterations of the Emmanoulopoulos-style loop, with inputs resident in HBM.

Default workload (PTF-like batch): 1024 curves of N = 2^14 samples, dt = 1 d,
per-curve Eq. 3 slopes a_low ~ U(0.8, 1.2), a_high ~ U(2, 3) and break
log-uniform in [1/1000, 1/50] per day, broken-power-law PDF draws of N values
per curve, 100 iterations in the FP32 form.

Prints one JSON line.  `value` = light-curve samples per second (curves x N
per step time).
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "light-curve samples/s through full iteration (FP32 batched vs FP64 plain); HBM %"

# MI355X published peaks
HBM_PEAK_GBS = 8000.0
LDS_PEAK_GBS = 256 * 128 * 2.4  # 256 CUs x 128 B/clk x 2.4 GHz = 78643 GB/s


def lds_bytes_per_sample_iter(n, prec_bytes):
    """LDS bytes one sample moves per iteration in the LDS-resident kernel:
    every FFT pass reads and writes the complex buffer (2 x prec bytes per
    real sample each way), the fold once, every radix pass writes and reads
    back the key and the 16-bit index and touches the packed digit counter
    (read + write + final read, 4 B each), and the final rank/scatter pass."""
    M = n // 2
    passes = 0
    m = M
    if m % 3 == 0:
        passes += 1
        m //= 3
    while m > 1:
        r = 8 if m % 8 == 0 else (4 if m % 4 == 0 else 2)
        passes += 1
        m //= r
    fft = 2 * passes * 2 * prec_bytes + 2 * prec_bytes
    key = prec_bytes
    npass = math.ceil(8 * key / 5)
    sort = npass * (2 * key + 2 * 2 + 3 * 4)
    post = 2 + 2 * 2 + prec_bytes
    return fft + sort + post


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="ptf_batch", choices=["ptf_batch", "single_curve"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run 5 device copies of 1 GiB (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        a = torch.empty(2**30, dtype=torch.uint8, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_launch": 2**30, "launches": 5}))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the generator shards "
              "independent curves across GPUs with no communication, which this build does not run.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1909_06374_amd as agn
    from paper_1909_06374_amd import synth

    dev = "cuda:0"
    if args.workload == "ptf_batch":
        n_curves, n, iters, prec = 1024, 2**14, 100, agn.AGN_FP32
        w = synth.ptf_batch(n_curves=n_curves, n=n, seed=1)
        params = [agn.psd_params(0.0, w["f_br"][c], w["a_low"][c], w["a_high"][c]) for c in range(n_curves)]
        erdf = w["erdf"].reshape(-1)
        desc = (f"ptf_batch: {n_curves} curves x N={n}, dt=1 d, per-curve Eq.3 slopes/break, "
                f"broken-power-law PDF draws, {iters} iterations, FP32 form")
    else:
        n_curves, n, iters, prec = 1, 1024, 50, agn.AGN_FP64
        w = synth.single_curve(n=n, seed=0)
        params = [agn.psd_params(**w["params"])]
        erdf = w["erdf"]
        desc = "single_curve: 1 curve x N=1024, dt=1 d, bending power law, 50 iterations, FP64"

    ns = [n] * n_curves
    offs = [c * n for c in range(n_curves)]
    seeds = [1000 + c for c in range(n_curves)]
    ids = list(range(n_curves))
    ctx = agn.Context(0)
    erdf_t = torch.as_tensor(erdf).to(dev)
    x = torch.empty(n_curves * n, dtype=torch.float64, device=dev)
    delta = torch.empty(n_curves * iters, dtype=torch.float64, device=dev)
    done = torch.empty(n_curves, dtype=torch.int32, device=dev)
    ws = torch.empty(agn.agn_batch_workspace_size(ns, prec), dtype=torch.uint8, device=dev)

    def step():
        agn.agn_lc_generate_batch(ctx, ns, offs, params, [1.0] * n_curves, [iters] * n_curves, seeds, ids,
                                  erdf_t, -1.0, prec, x, delta, done, ws)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ctx.kernel_times(reset=True)
    ctx.set_profiling(True)
    stream = torch.cuda.current_stream(dev)
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t0.record(stream)
    for _ in range(args.steps):
        step()
    t1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ctx.set_profiling(False)
    ms = t0.elapsed_time(t1) / args.steps
    kt = ctx.kernel_times(reset=True)
    assert int(done.min().item()) == iters, "a curve did not complete its iterations"

    samples = n_curves * n
    value = samples / (ms / 1000.0)
    dom = max(kt, key=lambda k: kt[k][0])
    dom_ms = kt[dom][0] / max(kt[dom][1], 1)
    pb = 4 if prec == agn.AGN_FP32 else 8
    per = lds_bytes_per_sample_iter(n, pb)
    lds_bytes = per * samples * iters
    achieved = lds_bytes / (dom_ms / 1000.0) / 1e9
    roof = {"bound": "lds", "kernel": dom, "achieved": round(achieved, 1), "peak": round(LDS_PEAK_GBS, 1),
            "unit": "GB/s", "frac": round(achieved / LDS_PEAK_GBS, 4), "traffic": None,
            "bytes_per_sample_iter": per, "avg_launch_ms": round(dom_ms, 4)}

    out = {
        "metric": METRIC, "value": value, "unit": "samples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32" if prec == agn.AGN_FP32 else "f64", "data": "synthetic",
        "config": {"workload": desc, "n_curves": n_curves, "n": n, "iters": iters,
                   "precision": "fp32" if prec == agn.AGN_FP32 else "fp64"},
        "sample_iterations_per_s": value * iters,
        "kernels_ms": {k: round(v[0] / max(v[1], 1), 4) for k, v in kt.items() if v[1]},
        "roofline": roof,
    }

    if not args.no_cpu_baseline:
        import oracle
        k = 4 if args.workload == "ptf_batch" else 1
        t = time.perf_counter()
        for c in range(k):
            op = oracle.psd_params(params[c].norm, params[c].f_br, params[c].a_low, params[c].a_high)
            oracle.generate(op, erdf[c * n:(c + 1) * n], 1.0, iters, seeds[c], ids[c])
        el = time.perf_counter() - t
        out["cpu_baseline"] = {"value": k * n / el, "unit": "samples/s", "cores": 1, "kind": "oracle",
                               "sample": f"first {k} curve(s) of the workload, all {iters} iterations, "
                                         f"single-threaded FP64 oracle ({el:.1f} s)"}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
