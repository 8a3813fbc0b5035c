"""Benchmark of the light-curve generator on one MI355X.

A step is one agn_lc_generate_batch call over the whole workload: Timmer-
Koenig moduli for every curve, the one-time sort of every PDF draw, and all
iterations of the Emmanoulopoulos-style loop, with inputs resident in HBM.

Default workload (long LSST-style curves): 4 curves of N = 2^26 samples,
dt = 7 d, Eq. 3 slopes (1, 2) with the break at 1/(10 yr), broken-power-law
PDF draws of N values per curve, 100 iterations in the FP32 form (FP64
twiddles and Eq. 4 sums); the same curves also run through the plain FP64
method, one curve per call, and the line reports both.

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
FP32_PEAK_TFLOPS = 157.3        # FP32 vector, packed FMA

# What the FP64 GPU path used as the reference here has been shown to equal.
REF_LABEL = ("FP64 GPU path: its permutation equals the FP64 oracle's for every length tested up to 2^16 and "
             "at sampled positions after one step at 2^20, 2^26 and 2^27")


def source_hash():
    """md5 (first 8 hex digits) of the HIP sources, in file-name order."""
    import glob
    import hashlib
    h = hashlib.md5()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_1909_06374_amd", "csrc", "*"))):
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:8]


def recorded_traffic(workload, kernel):
    """HBM bytes per launch of `kernel` from the rocprofv3 counter runs
    recorded in profiles/traffic.txt (FETCH_SIZE and WRITE_SIZE per dispatch,
    scaled by the copy calibration), or None if none is recorded or the HIP
    sources changed since the counters were taken."""
    kv, rows, _ = read_counters()
    if kv.get("sources") != source_hash() or (workload, kernel) not in rows:
        return None
    f, w = rows[(workload, kernel)]
    return (f * float(kv["fetch_scale"]) + w * float(kv["write_scale"])) * 1024.0


def read_counters():
    """profiles/traffic.txt as (settings, {(workload, kernel): (fetch KiB, write KiB)},
    {(workload, kernel): VALU instructions per launch})."""
    kv, rows, valu = {}, {}, {}
    path = os.path.join(ROOT, "profiles", "traffic.txt")
    if not os.path.exists(path):
        return kv, rows, valu
    for line in open(path):
        line = line.split("#", 1)[0].strip()
        if not line:
            continue
        parts = line.split()
        if len(parts) == 3 and parts[1] == "=":
            kv[parts[0]] = parts[2]
        elif len(parts) == 4 and parts[2] == "valu_insts":
            valu[(parts[0], parts[1])] = float(parts[3])
        elif len(parts) == 4:
            rows[(parts[0], parts[1])] = (float(parts[2]), float(parts[3]))
    return kv, rows, valu


def recorded_valu(workload, kernel):
    """VALU (wave64) instructions per launch of `kernel` from the rocprofv3
    SQ_INSTS_VALU run recorded in profiles/traffic.txt, or None if none is
    recorded or the HIP sources changed since."""
    kv, _, valu = read_counters()
    if kv.get("sources") != source_hash():
        return None
    return valu.get((workload, kernel))


def lds_flops_per_sample_iter(n):
    """FP32 flops per sample-iteration of the LDS-resident kernel counted
    algorithmically: the forward and the inverse real transform at
    2.5 N log2 N flops each, i.e. 5 log2 N per sample (70 at N = 2^14).  The
    modulus replacement (about 20 flops per sample) and the sort (integer
    work) are not counted, so the fraction understates how busy the kernel
    is; the LDS and VALU-issue views beside it say more."""
    return 5.0 * math.log2(n)


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


def hbm_bytes_per_sample(kernel, prec_bytes):
    """Algorithmic HBM bytes per real sample for one launch of a multi-pass
    kernel.  FFT pass: read and write the N/2-point complex buffer (prec bytes
    per real sample each way; the first forward pass reads more, so this is a
    lower bound for the average launch).  Sort scatter (8-bit LSD, key of prec
    bytes + 32-bit index): read key and index, write both; the first pass
    reads the key alone (the index is the position); the last pass instead
    reads the sorted value s[position] and writes x_{i+1}[sample].  Averaged
    over a sort's launches: (12 + 16 + 16 + 24) / 4 = 17 bytes in the FP32
    form, (20 + 6 x 24 + 28) / 8 = 24 in FP64.  Digit count (one launch per
    sort): read the key."""
    if kernel == "fft_pass":
        return 2 * prec_bytes
    if kernel == "sort_scatter":
        npass = prec_bytes
        move = 2 * (prec_bytes + 4)
        first = prec_bytes + prec_bytes + 4
        last = prec_bytes + 4 + 8 + 8
        return (first + move * (npass - 2) + last) / npass
    if kernel == "sort_hist":
        return prec_bytes
    if kernel in ("fold", "fft_mid"):
        # read and write the complex buffer, read the target moduli
        return 2 * prec_bytes + prec_bytes // 2
    return 8


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="lsst_long",
                    choices=["ptf_batch", "single_curve", "lsst_long", "lsst_long_fp64", "uneven_batch", "serving",
                             "paper_scale", "observables", "convergence", "pdf_draw"])
    ap.add_argument("--segment-iters", type=int, default=25,
                    help="serving: iterations per launch of a request (0: whole requests)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true", help="skip the FP32-vs-FP64 accuracy report")
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain FP64 run beside the FP32 form")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run 5 device copies of 1 GiB (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        a = torch.empty(2**30, dtype=torch.uint8, device="cuda:0")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(4):
            b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 4
        print(json.dumps({"copy_bytes_per_launch": 2**30, "launches": 5, "copy_ms": ms,
                          "copy_read_plus_write_gbs": 2 * 2**30 / (ms / 1000.0) / 1e9}))
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

    if args.workload == "uneven_batch":
        print(json.dumps(run_uneven(args, agn, synth, np, torch)))
        return
    if args.workload == "serving":
        print(json.dumps(run_serving(args, agn, np, torch)))
        return
    if args.workload == "observables":
        print(json.dumps(run_observables(args, agn, synth, np, torch)))
        return
    if args.workload == "convergence":
        print(json.dumps(run_convergence(args, agn, np, torch)))
        return
    if args.workload == "pdf_draw":
        print(json.dumps(run_pdf_draw(args, agn, np, torch)))
        return
    print(json.dumps(run_standard(args, agn, synth, np, torch)))


def cpu_info():
    """The host as the oracle baseline sees it: logical CPUs, the CPUs this
    process may run on, and the CPU model."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"nproc": os.cpu_count(), "usable_cpus": usable, "cpu_model": model}


def oracle_pool(jobs, threads):
    """Runs oracle calls (functions of no arguments) on `threads` host threads
    (the oracle's C calls release the GIL).  Returns the seconds each job took
    on its thread and the wall time of the whole pool."""
    from concurrent.futures import ThreadPoolExecutor

    def timed(f):
        t = time.perf_counter()
        f()
        return time.perf_counter() - t

    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        secs = list(ex.map(timed, jobs))
    return secs, time.perf_counter() - t0


def workload_setup(args, agn, synth, np):
    """(n_curves, n, iters, precision, PSD params, host draw or None, description, dt)."""
    if args.workload == "ptf_batch":
        n_curves, n, iters, prec = 1024, 2**14, 100, agn.AGN_FP32
        w = synth.ptf_batch(n_curves=n_curves, n=n, seed=1)
        params = [agn.psd_params(0.0, w["f_br"][c], w["a_low"][c], w["a_high"][c]) for c in range(n_curves)]
        erdf = w["erdf"].reshape(-1)
        desc = (f"ptf_batch: {n_curves} curves x N={n}, dt=1 d, per-curve Eq.3 slopes/break, "
                f"broken-power-law PDF draws, {iters} iterations, FP32 form")
        return n_curves, n, iters, prec, params, erdf, desc, 1.0
    if args.workload == "paper_scale":
        n_curves, n, iters, prec = 1, 2**27, 200, agn.AGN_FP64
        params = [agn.psd_params(0.0, 1.0 / (10 * synth.YEAR), 1.0, 2.0)]
        desc = ("paper_scale: 1 curve x N=2^27 (the paper's largest run), dt=7 d, Eq.3 slopes (1, 2), break "
                "1/(10 yr), broken-power-law PDF drawn on the device, 200 iterations, FP64")
        return n_curves, n, iters, prec, params, None, desc, 7.0
    if args.workload.startswith("lsst_long"):
        n_curves, n, iters = 4, 2**26, 100
        prec = agn.AGN_FP64 if args.workload.endswith("fp64") else agn.AGN_FP32
        params = [agn.psd_params(0.0, 1.0 / (10 * synth.YEAR), 1.0, 2.0)] * n_curves
        erdf = np.concatenate([synth.erdf_draw(n, seed=2, curve_id=c) for c in range(n_curves)])
        desc = (f"lsst_long: {n_curves} curves x N=2^26, dt=7 d (~1.29 Myr), Eq.3 slopes (1, 2), "
                f"break 1/(10 yr), broken-power-law PDF draws, {iters} iterations, "
                f"{'FP64' if prec == agn.AGN_FP64 else 'FP32 form (FP64 twiddles and Eq. 4 sums)'}")
        return n_curves, n, iters, prec, params, erdf, desc, 7.0
    n_curves, n, iters, prec = 1, 1024, 50, agn.AGN_FP64
    w = synth.single_curve(n=n, seed=0)
    params = [agn.psd_params(**w["params"])]
    desc = "single_curve: 1 curve x N=1024, dt=1 d, bending power law, 50 iterations, FP64"
    return n_curves, n, iters, prec, params, w["erdf"], desc, 1.0


def run_standard(args, agn, synth, np, torch):
    """One agn_lc_generate_batch call over the whole workload per step, timed
    without kernel instrumentation; per-kernel times come from one profiled
    repeat after the timed steps.  For the long-curve FP32 workload the same
    curves also run through the plain FP64 method, one curve per call."""
    dev = "cuda:0"
    n_curves, n, iters, prec, params, erdf, desc, dt_days = workload_setup(args, agn, synth, np)
    ns = [n] * n_curves
    offs = [c * n for c in range(n_curves)]
    seeds = [1000 + c for c in range(n_curves)]
    ids = list(range(n_curves))
    ctx = agn.Context(0)
    if erdf is None:
        erdf_t = torch.empty(n_curves * n, dtype=torch.float64, device=dev)
        for c in range(n_curves):
            agn.agn_erdf_draw(ctx, agn.erdf_params(), n, 27, c, erdf_t[c * n:(c + 1) * n])
        torch.cuda.synchronize()
    else:
        erdf_t = torch.as_tensor(erdf).to(dev)
    x = torch.empty(n_curves * n, dtype=torch.float64, device=dev)
    delta = torch.empty(n_curves * iters, dtype=torch.float64, device=dev)
    done = torch.empty(n_curves, dtype=torch.int32, device=dev)
    ws = torch.empty(agn.agn_batch_workspace_size(ns, prec), dtype=torch.uint8, device=dev)

    def step():
        agn.agn_lc_generate_batch(ctx, ns, offs, params, [dt_days] * n_curves, [iters] * n_curves, seeds,
                                  ids, erdf_t, -1.0, prec, x, delta, done, ws)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream(dev)
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for _ in range(args.steps):
        step()
    t1.record(stream)
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / args.steps
    assert int(done.min().item()) == iters, "a curve did not complete its iterations"

    # per-kernel times: one profiled repeat (events around every launch), kept
    # out of the timed steps
    ctx.kernel_times(reset=True)
    ctx.set_profiling(True)
    step()
    torch.cuda.synchronize()
    ctx.set_profiling(False)
    kt = ctx.kernel_times(reset=True)
    kt = {k: v for k, v in kt.items() if v[1]}

    samples = n_curves * n
    value = samples / (ms / 1000.0)
    dom = max(kt, key=lambda k: kt[k][0])
    dom_ms = kt[dom][0] / max(kt[dom][1], 1)
    pb = 4 if prec == agn.AGN_FP32 else 8
    if dom == "lds_iterate":
        # issue/barrier-bound: FP32 flops of the FFTs + replacement against the
        # vector peak; the LDS-traffic view alongside
        fl = lds_flops_per_sample_iter(n)
        achieved = fl * samples * iters / (dom_ms / 1000.0) / 1e12
        per = lds_bytes_per_sample_iter(n, pb)
        lds_gbs = per * samples * iters / (dom_ms / 1000.0) / 1e9
        # LDS ceiling measured on this device (agn_test_lds_bandwidth: 16-byte
        # conflict-free reads, 2048 workgroups x 4000 passes over 64 KB)
        probe = torch.empty(2048 * 1024, dtype=torch.float32, device=dev)
        lds_peak = agn.agn_test_lds_bandwidth(2048, 4000, probe) / 1e9
        roof = {"bound": "alu", "kernel": dom, "achieved": round(achieved, 3), "peak": FP32_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / FP32_PEAK_TFLOPS, 4),
                "traffic": recorded_traffic(args.workload, dom),
                "flops_per_sample_iter": fl, "avg_launch_ms": round(dom_ms, 4),
                "lds_view": {"achieved_gbs": round(lds_gbs, 1), "peak_gbs_measured": round(lds_peak, 1),
                             "frac": round(lds_gbs / lds_peak, 4), "bytes_per_sample_iter": per,
                             "peak_source": "agn_test_lds_bandwidth on this device"}}
        vi = recorded_valu(args.workload, dom)
        if vi is not None:
            # issue view: a wave64 VALU instruction holds a 16-lane SIMD for 4
            # cycles; 1024 SIMDs at 2.4 GHz
            cap = 1024 * 2.4e9 * (dom_ms / 1000.0) / 4.0
            roof["valu_issue_view"] = {"insts_per_launch": vi, "frac": round(vi / cap, 4),
                                       "source": "rocprofv3 SQ_INSTS_VALU, profiles/ptf_batch.md"}
    else:
        per = hbm_bytes_per_sample(dom, pb)
        achieved = per * samples / (dom_ms / 1000.0) / 1e9
        roof = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": recorded_traffic(args.workload, dom),
                "bytes_per_sample_per_launch": per, "avg_launch_ms": round(dom_ms, 4)}
        # whole step against the algorithmic bytes of one sample-iteration
        # (B_alg: 42 B in the FP32 form, 76 B in FP64)
        b_alg = 42 if prec == agn.AGN_FP32 else 76
        step_gbs = b_alg * samples * iters / (ms / 1000.0) / 1e9
        roof["step_view"] = {"bytes_per_sample_iter": b_alg, "achieved_gbs": round(step_gbs, 1),
                             "frac": round(step_gbs / HBM_PEAK_GBS, 4)}
    roof["traffic_source"] = ("recorded rocprofv3 FETCH_SIZE + WRITE_SIZE per launch (profiles/traffic.txt, "
                              "copy-calibrated) for these kernel sources" if roof["traffic"] is not None
                              else "no counter run recorded for these kernel sources")
    total_k = sum(v[0] for v in kt.values())
    out = {
        "metric": METRIC, "value": value, "unit": "samples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32" if prec == agn.AGN_FP32 else "f64", "data": "synthetic",
        "config": {"workload": desc, "n_curves": n_curves, "n": n, "iters": iters,
                   "precision": "fp32" if prec == agn.AGN_FP32 else "fp64"},
        "sample_iterations_per_s": value * iters,
        "hbm_bytes_alloc_gib": round((ws.numel() + x.numel() * 8 + erdf_t.numel() * 8) / 2**30, 2),
        "kernels_ms": {k: round(v[0] / max(v[1], 1), 4) for k, v in kt.items()},
        "kernel_time_share": {k: round(v[0] / total_k, 4) for k, v in kt.items()},
        "kernel_times_from": "one profiled repeat of the step after the timed steps",
        "roofline": roof,
    }

    x64 = None
    if args.workload == "lsst_long" and not args.no_fp64:
        # the plain method on the same curves: FP64, one agn_lc_generate call per curve
        ws64 = torch.empty(agn.agn_workspace_size(n, agn.AGN_FP64), dtype=torch.uint8, device=dev)
        x64 = torch.empty(n_curves * n, dtype=torch.float64, device=dev)
        done64 = torch.empty(n_curves, dtype=torch.int32, device=dev)

        def step64():
            for c in range(n_curves):
                agn.agn_lc_generate(ctx, params[c], erdf_t[c * n:(c + 1) * n], n, dt_days, iters, -1.0, seeds[c],
                                    ids[c], agn.AGN_FP64, x64[c * n:(c + 1) * n], None, done64[c:c + 1], ws64)

        step64()
        torch.cuda.synchronize()
        k64 = max(1, min(args.steps, 2))
        t0.record(stream)
        for _ in range(k64):
            step64()
        t1.record(stream)
        torch.cuda.synchronize()
        ms64 = t0.elapsed_time(t1) / k64
        assert int(done64.min().item()) == iters
        del ws64
        out["fp64_plain"] = {"ms_per_step": ms64, "value": samples / (ms64 / 1000.0), "unit": "samples/s",
                             "steps": k64, "warmup": 1,
                             "how": "the same curves in FP64, one agn_lc_generate call per curve"}
        out["speedup_fp32_vs_fp64_plain"] = ms64 / ms

    if prec == agn.AGN_FP32 and not args.no_accuracy and args.workload in ("ptf_batch", "lsst_long"):
        k = 8 if args.workload == "ptf_batch" else 1
        if args.workload == "ptf_batch":
            # the whole batch in FP64 for the ensemble statistic
            x64 = torch.empty_like(x)
            ws64 = torch.empty(agn.agn_batch_workspace_size(ns, agn.AGN_FP64), dtype=torch.uint8, device=dev)
            agn.agn_lc_generate_batch(ctx, ns, offs, params, [dt_days] * n_curves, [iters] * n_curves, seeds, ids,
                                      erdf_t, -1.0, agn.AGN_FP64, x64, None, None, ws64)
            del ws64
        out["accuracy_vs_fp64"] = fp32_accuracy(agn, np, torch, ctx, x, ns, offs, params, dt_days, iters,
                                                seeds, ids, erdf_t, k=k, x64_all=x64)
        if x64 is not None:
            out["accuracy_vs_fp64"]["ensemble_log_binned_periodogram_rel_diff_median_max"] = \
                ensemble_periodogram_diff(agn, np, torch, ctx, x, x64, ns, offs)

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = oracle_baseline(args, np, params, erdf, erdf_t, n, n_curves, dt_days, iters,
                                              seeds, ids)
    return out


def oracle_baseline(args, np, params, erdf, erdf_t, n, n_curves, dt_days, iters, seeds, ids):
    """The FP64 oracle on the host cores, parallel across curves only (one
    curve per thread; the per-curve code is the oracle as it stands).  Short
    curves run whole; long curves run a bounded piece: the first 2^21 samples
    of each curve at 1 and at 3 iterations, which separates the one-time work
    from the per-iteration cost; both are scaled to the full length by
    N log2 N and the step is extrapolated to all iterations."""
    import oracle
    info = cpu_info()
    if erdf is None:
        erdf = erdf_t[:min(erdf_t.numel(), n_curves * n)].cpu().numpy()
    op = [oracle.psd_params(p.norm, p.f_br, p.a_low, p.a_high) for p in params]
    if n > 2**20:
        ns_ = 2**21
        threads = max(1, min(n_curves, info["usable_cpus"] or 1))

        def job(c, it):
            return lambda: oracle.generate(op[c], erdf[c * n:c * n + ns_], dt_days, it, seeds[c], ids[c])

        jobs = [job(c, 1) for c in range(n_curves)] + [job(c, 3) for c in range(n_curves)]
        secs, wall = oracle_pool(jobs, threads)
        t1 = np.array(secs[:n_curves])
        t3 = np.array(secs[n_curves:])
        t_it = np.maximum((t3 - t1) / 2.0, 1e-9)
        t_once = np.maximum(t1 - t_it, 0.0)
        scale = (n / ns_) * (math.log2(n) / math.log2(ns_))
        step_s = float(np.max((t_once + iters * t_it) * scale)) * math.ceil(n_curves / threads)
        return {"value": n_curves * n / step_s, "unit": "samples/s", "cores": threads, "kind": "oracle",
                "extrapolated": True,
                "sample": f"first 2^21 samples of each of the {n_curves} curves at 1 and 3 iterations, one curve "
                          f"per thread ({wall:.1f} s wall); per-iteration and one-time costs scaled by N log2 N to "
                          f"N=2^{int(math.log2(n))} and to {iters} iterations",
                "oracle_step_s_extrapolated": round(step_s, 1),
                "single_thread_sample_iterations_per_s": float(np.mean(ns_ / t_it)),
                **info}
    k = min(n_curves, 8, info["usable_cpus"] or 1)
    threads = k

    def job(c):
        return lambda: oracle.generate(op[c], erdf[c * n:(c + 1) * n], dt_days, iters, seeds[c], ids[c])

    reps, secs_all, wall_all = 0, [], 0.0
    while True:  # at least one pass; repeated up to about 10 s of wall time
        secs, wall = oracle_pool([job(c) for c in range(k)], threads)
        secs_all += secs
        wall_all += wall
        reps += 1
        if wall_all >= 10.0:
            break
    return {"value": reps * k * n / wall_all, "unit": "samples/s", "cores": threads, "kind": "oracle",
            "sample": f"first {k} curve(s) of the workload, all {iters} iterations, one curve per thread, "
                      f"{reps} pass(es) ({wall_all:.1f} s wall)",
            "single_thread_samples_per_s": float(n / np.mean(secs_all)), **info}


def ensemble_periodogram_diff(agn, np, torch, ctx, x32, x64, ns, offs, dex=0.1):
    """Relative difference, bin by bin, of the mean 0.1-dex log-binned
    periodogram (Eq. A2) over all curves: FP32 form against FP64 (the
    ensemble statistic of Sec. 3.2.5).  Curves of one length only."""
    n, nc = ns[0], len(ns)
    nb = agn.agn_log_bin_count(n, dex)
    h = n // 2 + 1
    pws = torch.empty(agn.agn_periodogram_workspace_size(ns, dex), dtype=torch.uint8, device="cuda:0")
    P = torch.empty(nc * h, dtype=torch.float64, device="cuda:0")
    means = []
    for xx in (x32, x64):
        b = torch.empty(nc * nb, dtype=torch.float64, device="cuda:0")
        agn.agn_periodogram_batch(ctx, ns, offs, xx, [c * h for c in range(nc)], P, dex,
                                  [c * nb for c in range(nc)], b, pws)
        means.append(b.cpu().numpy().reshape(nc, nb).mean(axis=0))
    rel = np.abs(means[0] / means[1] - 1.0)
    return [float(np.median(rel)), float(rel.max())]


def log_binned_periodogram(np, x, dex=0.1):
    """Eq. A2 periodogram P_j = 2/N^2 |X_j|^2, j = 1..N/2, averaged in bins of
    `dex` in log10 frequency starting at the first Fourier frequency."""
    n = len(x)
    P = 2.0 / n**2 * np.abs(np.fft.rfft(x)[1:]) ** 2
    lj = np.log10(np.arange(1, n // 2 + 1))
    b = np.floor(lj / dex + 1e-9).astype(int)
    sums = np.bincount(b, weights=P)
    cnt = np.bincount(b)
    keep = cnt > 0
    return sums[keep] / cnt[keep]


def fp32_accuracy(agn, np, torch, ctx, x32_all, ns, offs, params, dt_days, iters, seeds, ids, erdf_t, k,
                  x64_all=None):
    """FP32 form against the FP64 path on the first k curves: value multiset,
    end-to-end and one-step rank agreement, |rank difference| quantiles,
    log-binned periodogram difference after all iterations and after one step
    from the same input.  x64_all: the FP64 run of the same curves, if made."""
    dev = "cuda:0"
    ns_k, offs_k = ns[:k], offs[:k]
    tot = int(sum(ns_k))
    if x64_all is not None:
        x64 = x64_all[:tot]
    else:
        x64 = torch.empty(tot, dtype=torch.float64, device=dev)
        ws = torch.empty(agn.agn_batch_workspace_size(ns_k, agn.AGN_FP64), dtype=torch.uint8, device=dev)
        agn.agn_lc_generate_batch(ctx, ns_k, offs_k, params[:k], [dt_days] * k, [iters] * k, seeds[:k], ids[:k],
                                  erdf_t[:tot], -1.0, agn.AGN_FP64, x64, None, None, ws)
        del ws
    torch.cuda.synchronize()
    a64 = x64.cpu().numpy()
    a32 = x32_all[:tot].cpu().numpy()
    multiset, e2e, one, drank, pdiff, pdiff1 = True, [], [], [], [], []
    for c in range(k):
        n, o = ns_k[c], offs_k[c]
        u32, u64 = a32[o:o + n], a64[o:o + n]
        s = np.sort(u64)
        multiset &= bool(np.array_equal(np.sort(u32), s))
        e2e.append(np.mean(u32 == u64))
        r32 = np.searchsorted(s, u32)
        r64 = np.searchsorted(s, u64)
        drank.append(np.abs(r32.astype(np.int64) - r64))
        p32, p64 = log_binned_periodogram(np, u32), log_binned_periodogram(np, u64)
        pdiff.append(np.abs(p32 / p64 - 1.0))
        # one step from the same input (the FP64 result) in both precisions
        ranks, outs = [], []
        for prec in (agn.AGN_FP32, agn.AGN_FP64):
            el = torch.float32 if prec == agn.AGN_FP32 else torch.float64
            amp = torch.empty(n // 2 + 1, dtype=el, device=dev)
            sws = torch.empty(agn.agn_spectrum_workspace_size(n), dtype=torch.uint8, device=dev)
            agn.agn_psd_spectrum(ctx, params[c], n, dt_days, seeds[c], ids[c], prec, amp, sws)
            iws = torch.empty(agn.agn_workspace_size(n, prec), dtype=torch.uint8, device=dev)
            xo = torch.empty(n, dtype=torch.float64, device=dev)
            rk = torch.empty(n, dtype=torch.int32, device=dev)
            agn.agn_lc_iterate(ctx, amp, x64[o:o + n], n, 1, -1.0, prec, xo, None, None, rk, iws)
            torch.cuda.synchronize()
            ranks.append(rk.cpu().numpy())
            outs.append(xo.cpu().numpy())
        one.append(np.mean(ranks[0] == ranks[1]))
        q32, q64 = log_binned_periodogram(np, outs[0]), log_binned_periodogram(np, outs[1])
        pdiff1.append(np.abs(q32 / q64 - 1.0))
    dr = np.concatenate(drank)
    pd = np.concatenate(pdiff)
    pd1 = np.concatenate(pdiff1)
    return {"curves": k, "reference": REF_LABEL,
            "value_multiset_exact": multiset,
            "one_step_rank_agreement": round(float(np.mean(one)), 6),
            "end_to_end_agreement": round(float(np.mean(e2e)), 6),
            "abs_rank_diff_p50_p99_max": [int(np.percentile(dr, 50)), int(np.percentile(dr, 99)), int(dr.max())],
            "log_binned_periodogram_rel_diff_median_max": [float(np.median(pd)), float(pd.max())],
            "one_step_log_binned_periodogram_rel_diff_median_max": [float(np.median(pd1)), float(pd1.max())]}


def run_uneven(args, agn, synth, np, torch):
    """Uneven batch: 8192 curves, lengths drawn uniformly from the 21 grid
    points 2^10..2^20 and 3 * 2^9..3 * 2^18, PTF-like per-curve PSD
    parameters, PDF draws made on the device (Philox stream 1), 100 FP32
    iterations.  The batch is a plan captured into a HIP graph with the
    number of concurrent launch chains chosen by the autotuner; a step is one
    graph launch."""
    dev = "cuda:0"
    n_curves, iters, prec, seed = 8192, 100, agn.AGN_FP32, 3
    ns = [int(v) for v in synth.uneven_sizes(n_curves, seed)]
    a_low, a_high, f_b = synth.curve_params(n_curves, seed)
    params = [agn.psd_params(0.0, f_b[c], a_low[c], a_high[c]) for c in range(n_curves)]
    offs = np.concatenate([[0], np.cumsum(ns)[:-1]]).astype(np.int64)
    total = int(np.sum(ns))
    ctx = agn.Context(0)
    erdf_t = torch.empty(total, dtype=torch.float64, device=dev)
    ep = agn.erdf_params()
    for c in range(n_curves):
        agn.agn_erdf_draw(ctx, ep, ns[c], seed, c, erdf_t[int(offs[c]):int(offs[c]) + ns[c]])
    x = torch.empty(total, dtype=torch.float64, device=dev)
    delta = torch.empty(n_curves * iters, dtype=torch.float64, device=dev)
    done = torch.empty(n_curves, dtype=torch.int32, device=dev)
    ws = torch.empty(agn.agn_batch_workspace_size(ns, prec), dtype=torch.uint8, device=dev)
    seeds = [1000 + c for c in range(n_curves)]
    ids = list(range(n_curves))
    t_plan = time.perf_counter()
    plan = agn.agn_batch_plan_create(ctx, ns, offs, params, [1.0] * n_curves, [iters] * n_curves, seeds, ids,
                                     erdf_t, -1.0, prec, x, delta, done,
                                     flags=agn.AGN_PLAN_GRAPH | agn.AGN_PLAN_AUTOTUNE, ws=ws)
    torch.cuda.synchronize()
    t_plan = time.perf_counter() - t_plan
    info = plan.info()
    stream = torch.cuda.current_stream(dev)
    for _ in range(args.warmup):
        agn.agn_batch_plan_launch(plan)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for _ in range(args.steps):
        agn.agn_batch_plan_launch(plan)
    t1.record(stream)
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / args.steps
    assert int(done.min().item()) == iters, "a curve did not complete its iterations"
    # kernel breakdown: one eager (non-graph) profiled run after the timed steps
    ctx.kernel_times(reset=True)
    ctx.set_profiling(True)
    agn.agn_lc_generate_batch(ctx, ns, offs, params, [1.0] * n_curves, [iters] * n_curves, seeds, ids,
                              erdf_t, -1.0, prec, x, delta, done, ws)
    torch.cuda.synchronize()
    ctx.set_profiling(False)
    kt = ctx.kernel_times(reset=True)
    value = total / (ms / 1000.0)
    dom = max(kt, key=lambda k: kt[k][0])
    dom_ms = kt[dom][0] / max(kt[dom][1], 1)
    share = {k: round(v[0] / sum(u[0] for u in kt.values()), 4) for k, v in kt.items() if v[1]}
    out = {
        "metric": METRIC, "value": value, "unit": "samples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"uneven_batch: {n_curves} curves, N uniform over the 21 lengths 2^10..2^20 and "
                               f"3*2^9..3*2^18 (sum N = {total}), PTF-like per-curve Eq.3 parameters, device PDF "
                               f"draws, {iters} iterations, FP32 form, HIP-graph plan",
                   "n_curves": n_curves, "sum_n": total, "iters": iters, "precision": "fp32"},
        "sample_iterations_per_s": value * iters,
        "plan": dict(info, create_s=round(t_plan, 2)),
        "hbm_bytes_alloc_gib": round((ws.numel() + x.numel() * 8 + erdf_t.numel() * 8) / 2**30, 2),
        "kernel_time_share_eager": share,
        "roofline": {"bound": "hbm" if dom != "lds_iterate" else "alu", "kernel": dom,
                     "avg_launch_ms": round(dom_ms, 4), "note": "per-kernel times from one eager profiled run"},
    }
    if dom == "sort_scatter":
        # algorithmic bytes of every scatter launch of the eager run: multi-pass
        # curves only; per iteration 4 passes of 32-bit keys (17 bytes per key on
        # average), once 8 passes of the 64-bit draw keys (2 (8 + 4) bytes per key)
        big = [nn for nn in ns if not ((nn % 3 == 0 and nn <= 12288) or (nn % 3 != 0 and nn <= 16384))]
        byts = float(sum(big)) * (iters * 4 * hbm_bytes_per_sample("sort_scatter", 4) + 8 * 24)
        achieved = byts / (kt[dom][0] / 1000.0) / 1e9
        out["roofline"].update({"achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                                "bytes": "17 per key per pass on average (FP32 keys; the first pass reads the "
                                         "key alone, the last reads s[position] and writes x), 24 for the one-time "
                                         "draw sort"})
    if not args.no_cpu_baseline:
        import oracle
        # bounded sample: the first curves of the batch up to 2^21 samples, 3 iterations
        # each, scaled per sample-iteration to the full iteration count
        k, acc = 0, 0
        while acc < 2**21:
            acc += ns[k]
            k += 1
        it_ = 3
        host_erdf = erdf_t[:acc].cpu().numpy()
        t = time.perf_counter()
        for c in range(k):
            op = oracle.psd_params(0.0, float(f_b[c]), float(a_low[c]), float(a_high[c]))
            oracle.generate(op, host_erdf[int(offs[c]):int(offs[c]) + ns[c]], 1.0, it_, seeds[c], ids[c])
        el = time.perf_counter() - t
        out["cpu_baseline"] = {"value": acc * it_ / el / iters, "unit": "samples/s", "cores": 1, "kind": "oracle",
                               "sample": f"first {k} curves ({acc} samples) x {it_} iterations of the "
                                         f"single-threaded FP64 oracle ({el:.1f} s), scaled per "
                                         f"sample-iteration to {iters} iterations"}
    plan.close()
    return out


def run_serving(args, agn, np, torch):
    """Request serving: Poisson arrivals, N uniform over the 2^a / 3 * 2^a grid
    in [2^12, 2^22], 50-200 iterations, PTF-like PSD parameters, FP32 form,
    continuous batching over 4 streams with HBM-footprint admission.
    Capacity = request rate served with every request queued at time zero;
    then a load sweep at 25/50/75/100% of capacity and the specified 2000/s
    offered load (each over a bounded arrival window); `value` is the
    saturated throughput in samples/s.  Baseline: FP64, one request at a time."""
    from paper_1909_06374_amd.serving import GpuBackend, Request, Server, make_requests
    ctx = agn.Context(0)
    free, _ = torch.cuda.mem_get_info(0)
    budget = int(min(0.6 * free, 160 * 2**30))
    be = GpuBackend(ctx, n_slots=4, prec=agn.AGN_FP32)
    # iteration-level batching: a launch runs at most `seg` iterations of a
    # request, so later arrivals join at the next segment boundary
    seg = args.segment_iters if args.segment_iters > 0 else None
    srv = Server(be, budget_bytes=budget, segment_iters=seg)
    # warm-up: one small request of each path
    srv.run([Request(rid=10**6 + i, n=n, iters=3, f_br=0.01, a_low=1.0, a_high=2.0, seed=i, arrival=0.0)
             for i, n in enumerate([4096, 2**20])])
    base = make_requests(rate_hz=2000.0, duration_s=60.0, seed=4)
    n_cap = 192
    cap_reqs = [Request(**{**r.__dict__, "arrival": 0.0}) for r in base[:n_cap]]
    st = srv.run(cap_reqs)
    cap_rps = st.completed / max(r.done for r in cap_reqs)
    cap_sps = st.samples / max(r.done for r in cap_reqs)
    # kernel shares from a second, profiled run of the same requests (kernel
    # timing adds events around every launch, so it is kept out of the timed run)
    prof_reqs = [Request(**{**r.__dict__, "arrival": 0.0}) for r in base[:n_cap]]
    ctx.kernel_times(reset=True)
    ctx.set_profiling(True)
    srv.run(prof_reqs)
    torch.cuda.synchronize()
    ctx.set_profiling(False)
    kt = ctx.kernel_times(reset=True)
    kt = {k: v for k, v in kt.items() if v[1] and k != "batch_graph"}
    dom = max(kt, key=lambda k: kt[k][0])
    roof = {"bound": "hbm" if dom != "lds_iterate" else "alu", "kernel": dom,
            "avg_launch_ms": round(kt[dom][0] / kt[dom][1], 4), "traffic": None,
            "kernel_time_share": {k: round(v[0] / sum(u[0] for u in kt.values()), 4) for k, v in kt.items()},
            "note": "kernel times of a profiled repeat of the capacity run (all requests queued at once)"}
    if dom == "sort_scatter":
        # multi-pass requests: per iteration 4 passes of 32-bit keys (17 bytes per
        # key on average), once 8 passes of the 64-bit draw keys (24 bytes per key)
        big = [r for r in cap_reqs if not ((r.n % 3 == 0 and r.n <= 12288) or (r.n % 3 != 0 and r.n <= 16384))]
        # (the draw keys are sorted once per segment)
        nseg = [1 if seg is None else -(-r.iters // seg) for r in big]
        per = hbm_bytes_per_sample("sort_scatter", 4)
        byts = float(sum(r.n * (r.iters * 4 * per + k * 8 * 24) for r, k in zip(big, nseg)))
        ach = byts / (kt[dom][0] / 1000.0) / 1e9
        roof.update({"achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(ach / HBM_PEAK_GBS, 4)})
    sweep = []
    window = 6.0
    for frac in (0.25, 0.5, 0.75, 1.0):
        rate = frac * cap_rps
        reqs = make_requests(rate_hz=rate, duration_s=window, seed=40 + int(100 * frac))
        if not reqs:
            continue
        st = srv.run(reqs)
        span = max(r.done for r in reqs)
        sweep.append({"offered_frac_of_capacity": frac, "offered_req_per_s": round(rate, 2),
                      "requests": st.completed, "p50_latency_s": round(st.latency_p50_s, 4),
                      "p99_latency_s": round(st.latency_p99_s, 4), "samples_per_s": st.samples / span,
                      "batches": st.batches, "mean_batch": round(st.mean_batch, 2)})
        print(f"serving sweep {frac:.2f}: p50 {st.latency_p50_s:.3f} s p99 {st.latency_p99_s:.3f} s",
              file=sys.stderr, flush=True)
    spec_window = 1.0
    reqs = make_requests(rate_hz=2000.0, duration_s=spec_window, seed=4)
    st = srv.run(reqs)
    span = max(r.done for r in reqs)
    spec = {"offered_req_per_s": 2000.0, "arrival_window_s": spec_window, "requests": st.completed,
            "p50_latency_s": round(st.latency_p50_s, 4), "p99_latency_s": round(st.latency_p99_s, 4),
            "samples_per_s": st.samples / span, "max_footprint_gib": round(st.max_footprint / 2**30, 2)}
    # FP64 one request at a time
    k = 6
    one = base[:k]
    ws = None
    t_ev0 = torch.cuda.Event(enable_timing=True)
    t_ev1 = torch.cuda.Event(enable_timing=True)
    bufs = []
    for r in one:
        e = torch.empty(r.n, dtype=torch.float64, device="cuda:0")
        agn.agn_erdf_draw(ctx, agn.erdf_params(), r.n, r.seed, r.rid, e)
        bufs.append(e)
    mx = max(r.n for r in one)
    ws = torch.empty(agn.agn_workspace_size(mx, agn.AGN_FP64), dtype=torch.uint8, device="cuda:0")
    xo = torch.empty(mx, dtype=torch.float64, device="cuda:0")
    torch.cuda.synchronize()
    t_ev0.record()
    for r, e in zip(one, bufs):
        agn.agn_lc_generate(ctx, agn.psd_params(0.0, r.f_br, r.a_low, r.a_high), e, r.n, 1.0, r.iters, -1.0,
                            r.seed, r.rid, agn.AGN_FP64, xo[:r.n], None, None, ws)
        torch.cuda.synchronize()
    t_ev1.record()
    torch.cuda.synchronize()
    el = t_ev0.elapsed_time(t_ev1) / 1000.0
    fp64 = {"requests": k, "req_per_s": k / el, "samples_per_s": sum(r.n for r in one) / el,
            "sample": f"first {k} requests of the 2000/s stream, FP64, one agn_lc_generate call each"}
    # the same requests through the server (FP32 form, all queued at time zero)
    same = [Request(**{**r.__dict__, "arrival": 0.0, "rid": r.rid}) for r in one]
    st_same = srv.run(same)
    span_same = max(r.done for r in same)
    fp64["fp32_served_same_requests_req_per_s"] = st_same.completed / span_same
    fp64["speedup_fp32_served_vs_fp64_one_at_a_time"] = (st_same.completed / span_same) / (k / el)
    return {
        "metric": METRIC, "value": cap_sps, "unit": "samples/s", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": 1000.0 / cap_rps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "serving: Poisson arrivals, N uniform over 2^12..2^22 (2^a and 3*2^a), 50-200 "
                               "iterations, PTF-like PSD parameters, device PDF draws, FP32 form, 4 streams, "
                               "HBM-footprint admission, " + (f"segments of {seg} iterations" if seg else
                                                               "whole requests per launch"),
                   "budget_gib": round(budget / 2**30, 1), "segment_iters": seg},
        "capacity_req_per_s": cap_rps, "capacity_requests": n_cap,
        "load_sweep": sweep, "offered_2000_per_s": spec, "fp64_one_at_a_time": fp64,
        "roofline": roof, "cpu_baseline": serving_cpu_baseline(args, base),
    }


def serving_cpu_baseline(args, reqs):
    """The FP64 oracle on the first requests of the stream with N <= 2^16, each
    at its own iteration count, for about 5 s (samples/s of whole requests)."""
    if args.no_cpu_baseline:
        return None
    import oracle
    from paper_1909_06374_amd import synth
    t = time.perf_counter()
    done, samples = 0, 0
    for r in reqs:
        if r.n > 2**16:
            continue
        erdf = synth.erdf_draw(r.n, seed=r.seed, curve_id=r.rid)
        oracle.generate(oracle.psd_params(0.0, r.f_br, r.a_low, r.a_high), erdf, 1.0, r.iters, r.seed, r.rid)
        done += 1
        samples += r.n
        if time.perf_counter() - t >= 5.0:
            break
    el = time.perf_counter() - t
    return {"value": samples / el, "unit": "samples/s", "cores": 1, "kind": "oracle",
            "sample": f"{done} requests of the stream with N <= 2^16, each at its own 50-200 iterations, "
                      f"single-threaded FP64 oracle ({el:.1f} s)"}


def run_observables(args, agn, synth, np, torch):
    """Observables of the PTF-like batch's output (1024 curves x 2^14, FP32
    form, 100 iterations; generated once, untimed): one step is the
    periodogram of Eq. A2 with 0.1-dex bins, plus the lag statistics at 40
    log-spaced lags in magnitudes -- Eq. A6 SF^2, its Eq. 6 mean over the
    curves, and counts of |dm| above 6 thresholds with Table 2's cut
    log lambda = -1.2 (Figs. 16-17)."""
    dev = "cuda:0"
    n_curves, n, iters = 1024, 2**14, 100
    w = synth.ptf_batch(n_curves=n_curves, n=n, seed=1)
    params = [agn.psd_params(0.0, w["f_br"][c], w["a_low"][c], w["a_high"][c]) for c in range(n_curves)]
    ns = [n] * n_curves
    offs = [c * n for c in range(n_curves)]
    ctx = agn.Context(0)
    erdf_t = torch.as_tensor(w["erdf"].reshape(-1)).to(dev)
    x = torch.empty(n_curves * n, dtype=torch.float64, device=dev)
    ws = torch.empty(agn.agn_batch_workspace_size(ns, agn.AGN_FP32), dtype=torch.uint8, device=dev)
    agn.agn_lc_generate_batch(ctx, ns, offs, params, [1.0] * n_curves, [iters] * n_curves,
                              [1000 + c for c in range(n_curves)], list(range(n_curves)), erdf_t, -1.0,
                              agn.AGN_FP32, x, None, None, ws)
    del ws
    dex = 0.1
    h = n // 2 + 1
    nb = agn.agn_log_bin_count(n, dex)
    P = torch.empty(n_curves * h, dtype=torch.float64, device=dev)
    bins = torch.empty(n_curves * nb, dtype=torch.float64, device=dev)
    pws = torch.empty(agn.agn_periodogram_workspace_size(ns, dex), dtype=torch.uint8, device=dev)
    lags = np.unique(np.round(np.logspace(0, np.log10(n // 2), 40)).astype(np.int64))
    dm = [0.1, 0.25, 0.5, 1.0, 2.5, 5.0]
    cut = 10.0 ** -1.2
    K, J = len(lags), len(dm)
    sf2 = torch.empty(n_curves * K, dtype=torch.float64, device=dev)
    rep = torch.empty(K, dtype=torch.float64, device=dev)
    ex = torch.empty(n_curves * K * J, dtype=torch.int64, device=dev)
    pairs = torch.empty(n_curves * K, dtype=torch.int64, device=dev)
    lws = torch.empty(agn.agn_lag_stats_workspace_size(ns, lags, J, agn.AGN_SF_MAGNITUDE), dtype=torch.uint8, device=dev)

    def step():
        agn.agn_periodogram_batch(ctx, ns, offs, x, [c * h for c in range(n_curves)], P, dex,
                                  [c * nb for c in range(n_curves)], bins, pws)
        agn.agn_lag_stats_batch(ctx, ns, offs, x, lags, agn.AGN_SF_MAGNITUDE, sf2, rep, dm, cut, ex, pairs, lws)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ctx.kernel_times(reset=True)
    ctx.set_profiling(True)
    stream = torch.cuda.current_stream(dev)
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record(stream)
    for _ in range(args.steps):
        step()
    t1.record(stream)
    torch.cuda.synchronize()
    ctx.set_profiling(False)
    ms = t0.elapsed_time(t1) / args.steps
    kt = ctx.kernel_times(reset=True)
    samples = n_curves * n
    pairs_per_step = int(sum(n - k for k in lags)) * n_curves
    dom = max(kt, key=lambda k: kt[k][0])
    dom_ms = kt[dom][0] / max(kt[dom][1], 1)
    if dom == "lag_stats":
        # algorithmic bytes: each lag reads the series once (8 B per pair)
        per = 8.0
        achieved = per * pairs_per_step / (dom_ms / 1000.0) / 1e9
        unit_note = "bytes_per_pair"
    else:
        # periodogram: read x once, write P once
        per = 8.0 + 4.0
        achieved = per * samples / (dom_ms / 1000.0) / 1e9
        unit_note = "bytes_per_sample"
    roof = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": recorded_traffic(args.workload, dom),
            unit_note: per, "avg_launch_ms": round(dom_ms, 4)}
    out = {
        "metric": "light-curve samples/s through the observables (Eq. A2 periodogram + Eq. A6 SF + |dm| counts)",
        "value": samples / (ms / 1000.0), "unit": "samples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"observables of the PTF-like batch output: {n_curves} curves x N={n}; periodogram "
                               f"with {dex}-dex bins; SF^2 in magnitudes at {K} log-spaced lags 1..{n // 2} with "
                               f"the Eq. 6 mean; |dm| counts over {J} thresholds with cut log lambda = -1.2",
                   "n_curves": n_curves, "n": n, "lags": K, "thresholds": J},
        "pairs_per_s": pairs_per_step / (ms / 1000.0),
        "kernels_ms": {k: round(v[0] / max(v[1], 1), 4) for k, v in kt.items() if v[1]},
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        import oracle
        k = 384  # about 10 s of single-threaded oracle work
        xh = x[:k * n].cpu().numpy()
        t = time.perf_counter()
        for c in range(k):
            xc = xh[c * n:(c + 1) * n]
            oracle.log_binned(oracle.periodogram(xc), n, 1.0, dex)
            oracle.lag_stats(xc, lags, 1, dm, cut)
        el = time.perf_counter() - t
        out["cpu_baseline"] = {"value": k * n / el, "unit": "samples/s", "cores": 1, "kind": "oracle",
                               "sample": f"first {k} curves, the same observables, single-threaded FP64 oracle "
                                         f"({el:.1f} s)"}
    return out


def run_convergence(args, agn, np, torch):
    """Validation workload: the convergence test of Sec. 3.2.2 (Eq. 3 fitted
    to each curve's log-binned periodogram, fitted slopes followed over the
    iterations) and the collapse of Sec. 3.2.9 (a 6-dex W17 PDF with steep
    single power laws), next to Eq. 4's distance.  Iterations run in segments:
    a segment restarts the generator from the previous output, which is a
    permutation of the same draw, so its sorted values and the spectrum (same
    seeds) are unchanged and the run continues exactly."""
    dev = "cuda:0"
    ctx = agn.Context(0)
    n, nc, dex = 2**16, 32, 0.1
    checkpoints = [1, 2, 5, 10, 20, 50, 100, 200]
    fb = 1.0 / 1000.0
    w17 = dict(u_star=-1.84, d1=0.47, d2=2.53)
    setups = [
        ("table2_pdf_bending_psd", agn.pdf_params(agn.AGN_PDF_EQ1), (1.0, 2.0)),
        ("w17_pdf_6dex_alpha1.6", agn.pdf_params(agn.AGN_PDF_EQ1, u_min=-5.0, u_max=1.0, **w17), (1.6, 1.6)),
        ("w17_pdf_6dex_alpha1.8", agn.pdf_params(agn.AGN_PDF_EQ1, u_min=-5.0, u_max=1.0, **w17), (1.8, 1.8)),
        ("w17_pdf_6dex_alpha2.0", agn.pdf_params(agn.AGN_PDF_EQ1, u_min=-5.0, u_max=1.0, **w17), (2.0, 2.0)),
        ("w17_pdf_2dex_alpha2.0", agn.pdf_params(agn.AGN_PDF_EQ1, u_min=-2.84, u_max=-0.84, **w17), (2.0, 2.0)),
    ]
    ns = [n] * nc
    offs = [c * n for c in range(nc)]
    nb = agn.agn_log_bin_count(n, dex)
    P = torch.empty(nc * (n // 2 + 1), dtype=torch.float64, device=dev)
    bins = torch.empty(nc * nb, dtype=torch.float64, device=dev)
    fit = torch.empty(nc * 4, dtype=torch.float64, device=dev)
    pws = torch.empty(agn.agn_periodogram_workspace_size(ns, dex), dtype=torch.uint8, device=dev)
    fws = torch.empty(agn.agn_psd_fit_workspace_size(ns, dex), dtype=torch.uint8, device=dev)
    gws = torch.empty(agn.agn_batch_workspace_size(ns, agn.AGN_FP64), dtype=torch.uint8, device=dev)
    xa = torch.empty(nc * n, dtype=torch.float64, device=dev)
    xb = torch.empty_like(xa)
    delta = torch.empty(nc * checkpoints[-1], dtype=torch.float64, device=dev)
    done = torch.empty(nc, dtype=torch.int32, device=dev)
    results = {}
    t_an = 0.0
    n_an = 0
    for name, pdf, (al, ah) in setups:
        params = [agn.psd_params(0.0, fb, al, ah)] * nc
        for c in range(nc):
            agn.agn_pdf_draw(ctx, pdf, n, 77, c, xa[c * n:(c + 1) * n])
        rows = []
        it = 0
        for cp in checkpoints:
            seg = cp - it
            agn.agn_lc_generate_batch(ctx, ns, offs, params, [1.0] * nc, [seg] * nc, [500 + c for c in range(nc)],
                                      list(range(nc)), xa, -1.0, agn.AGN_FP64, xb, delta, done, gws)
            last_delta = delta[:nc * seg].view(nc, seg)[:, seg - 1].cpu().numpy()
            xa, xb = xb, xa
            it = cp
            torch.cuda.synchronize()
            ctx.set_profiling(True)
            t = time.perf_counter()
            agn.agn_periodogram_batch(ctx, ns, offs, xa, [c * (n // 2 + 1) for c in range(nc)], P, dex,
                                      [c * nb for c in range(nc)], bins, pws)
            agn.agn_psd_fit_batch(ctx, ns, [1.0] * nc, params, dex, [c * nb for c in range(nc)], bins, fit, fws)
            torch.cuda.synchronize()
            t_an += time.perf_counter() - t
            ctx.set_profiling(False)
            n_an += nc
            f = fit.view(nc, 4).cpu().numpy()
            mean_slope = 0.5 * (f[:, 1] + f[:, 2])
            collapsed = (np.abs(mean_slope - 1.0) < 0.25) & (f[:, 3] < 0.1)
            rows.append({"iteration": cp, "a_low_median": round(float(np.median(f[:, 1])), 3),
                         "a_high_median": round(float(np.median(f[:, 2])), 3),
                         "rms_median": round(float(np.median(f[:, 3])), 4),
                         "delta_median": float(np.median(last_delta)),
                         "collapsed_fraction": round(float(np.mean(collapsed)), 3)})
        results[name] = {"input_slopes": [al, ah], "checkpoints": rows}
    kt = {k: v for k, v in ctx.kernel_times(reset=True).items() if v[1]}
    pg_ms = kt.get("periodogram", (0.0, 0))[0]
    # periodogram launches: read the series (8 B) and write P (4 B per sample)
    ach = 12.0 * n * n_an / (pg_ms / 1000.0) / 1e9 if pg_ms > 0 else None
    roof = {"bound": "hbm", "kernel": "periodogram", "achieved": None if ach is None else round(ach, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": None if ach is None else round(ach / HBM_PEAK_GBS, 4),
            "traffic": None, "kernels_ms_total": {k: round(v[0], 3) for k, v in kt.items()},
            "note": "the fit runs one wave per curve and is latency-bound"}
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        xh = xa[:4 * n].cpu().numpy()
        t = time.perf_counter()
        for c in range(4):
            fm, pm = oracle.log_binned_mean_f(oracle.periodogram(xh[c * n:(c + 1) * n]), n, 1.0, dex)
            oracle.psd_fit(fm, pm, fb, 2.0, 2.0)
        el = time.perf_counter() - t
        cpu = {"value": 4 / el, "unit": "curve fits/s", "cores": 1, "kind": "oracle",
               "sample": f"periodogram, bins and fit of 4 curves of the last setup ({el:.2f} s)"}
    return {
        "metric": "E13 convergence test: Eq. 3 fits of log-binned periodograms per curve (validation workload)",
        "value": n_an / t_an, "unit": "curve fits/s (periodogram + bins + fit, host-timed)", "n_gpus": 1,
        "steps": len(setups) * len(checkpoints), "warmup": 0, "ms_per_step": 1000.0 * t_an / (n_an / nc),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{nc} curves x N=2^16 per setup, FP64, Eq. 1 PDF draws on the device, Eq. 3 "
                               f"with the break at 1/1000 d^-1, fits at iterations {checkpoints}; collapse "
                               f"flagged where the mean fitted slope is within 0.25 of 1 and the rms of the "
                               f"log10 residuals is below 0.1",
                   "n_curves": nc, "n": n},
        "setups": results, "roofline": roof, "cpu_baseline": cpu,
    }


def run_pdf_draw(args, agn, np, torch):
    """The PDF draw of Sec. 2.1 step (ii) at the long-curve size: 2^26 draws of
    Table 2's Eq. 1 PDF read as dN/dlambda, by the exact inverse CDF
    (agn_pdf_draw) and by the paper's slice sampling in linear lambda
    (agn_pdf_slice on 2^22 draws: 2^18 chains of 16 draws after 200 steps of
    burn-in; burn-in included in its time)."""
    dev = "cuda:0"
    ctx = agn.Context(0)
    n = 2**26
    p = agn.pdf_params(agn.AGN_PDF_EQ1, agn.AGN_PDF_PER_LINEAR)
    out = torch.empty(n, dtype=torch.float64, device=dev)
    chains, burn, n_slice = 2**18, 200, 2**22

    def timed(f, reps):
        f()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            f()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    ms_inv = timed(lambda: agn.agn_pdf_draw(ctx, p, n, 1, 0, out), max(args.steps, 3))
    ms_slice = timed(lambda: agn.agn_pdf_slice(ctx, p, n_slice, chains, burn, 1, 0, out), 1)
    gbs = 8.0 * n / (ms_inv / 1000.0) / 1e9
    res = {
        "metric": "PDF draws/s (Sec. 2.1 step ii), inverse CDF on the device", "value": n / (ms_inv / 1000.0),
        "unit": "draws/s", "n_gpus": 1, "steps": max(args.steps, 3), "warmup": 1, "ms_per_step": ms_inv,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "2^26 draws of Table 2's Eq. 1 PDF (lambda* = 0.11, slopes 0.47 / 2.53, "
                               "log lambda in [-3.75, 0.5]) read as dN/dlambda", "n": n},
        "roofline": {"bound": "hbm", "kernel": "erdf_draw (k_pdf_eq1)", "achieved": round(gbs, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None,
                     "bytes_per_draw": 8, "avg_launch_ms": round(ms_inv, 4)},
        "slice_sampling": {"draws": n_slice, "ms": ms_slice, "draws_per_s": n_slice / (ms_slice / 1000.0),
                           "chains": chains, "burn": burn, "steps_per_chain": burn + n_slice // chains},
    }
    if not args.no_cpu_baseline:
        import oracle
        op = oracle.pdf_params(1, 1)
        k = 400000
        t = time.perf_counter()
        oracle.pdf_draw(op, k, 1, 0)
        el = time.perf_counter() - t
        res["cpu_baseline"] = {"value": k / el, "unit": "draws/s", "cores": 1, "kind": "oracle",
                               "sample": f"{k} inverse-CDF draws of the single-threaded FP64 oracle ({el:.1f} s)"}
    return res


if __name__ == "__main__":
    main()
