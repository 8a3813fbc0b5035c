"""Writes tests/golden/one_step_2p26.json and one_step_2p27.json from the CPU
oracle only: one iteration (Sec. 2.1) of the long curves at sampled samples.

Workloads (inputs from paper_1909_06374_amd.synth, the seeded generators):
  2^26: the long LSST-style curve -- N = 2^26, dt = 7 d, Eq. 3 slopes (1, 2),
        break 1/(10 yr) = 1/3652.5 per day, unit-variance normalisation,
        the broken-power-law PDF draw (synth.erdf_draw seed 2, curve 0),
        Timmer-Koenig moduli with Philox seed 1000, curve 0.
  2^27: the paper's largest run (Sec. 3.2.3) with the same PSD, PDF draw
        synth.erdf_draw seed 27, curve 0, moduli seed 1000, curve 0.
For 4096 sample indices t drawn by numpy's Philox (seed 7) the file holds the
oracle's rank of sample t after one iteration and the gap of y[t] to its
nearest neighbour in sorted order, relative to rms(y) (y = the inverse
transform the step ranks); plus delta_1 of Eq. 4.  Runs take minutes.
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_1909_06374_amd import synth  # noqa: E402

CASES = {
    26: dict(n=2**26, erdf_seed=2),
    27: dict(n=2**27, erdf_seed=27),
}
DT = 7.0
F_BR = 1.0 / 3652.5
SAMPLES = 4096


def sample_indices(n):
    return np.sort(np.random.Generator(np.random.Philox(7)).integers(0, n, SAMPLES)).astype(np.int64)


def make(lg):
    c = CASES[lg]
    n = c["n"]
    x0 = synth.erdf_draw(n, seed=c["erdf_seed"], curve_id=0)
    p = oracle.psd_params(0.0, F_BR, 1.0, 2.0)
    amp = oracle.psd_spectrum(p, n, DT, 1000, 0)
    _, delta, done, rank = oracle.iterate(amp, x0, 1)
    y = oracle.irfft(oracle.replace(oracle.rfft(x0), amp, n), n)
    rms = float(np.sqrt(np.mean(y * y)))
    ys = np.sort(y)
    idx = sample_indices(n)
    k = rank[idx].astype(np.int64)
    lo = np.where(k > 0, ys[k] - ys[np.maximum(k - 1, 0)], np.inf)
    hi = np.where(k < n - 1, ys[np.minimum(k + 1, n - 1)] - ys[k], np.inf)
    gap = np.minimum(lo, hi) / rms
    out = {
        "workload": f"N=2^{lg}, dt=7 d, Eq.3 slopes (1, 2), f_br=1/3652.5 d^-1, unit variance; "
                    f"PDF draw synth.erdf_draw(seed={c['erdf_seed']}, curve 0); moduli seed 1000 curve 0; "
                    "one iteration of the FP64 oracle",
        "n": n, "erdf_seed": c["erdf_seed"], "spectrum_seed": 1000, "curve_id": 0, "dt": DT, "f_br": F_BR,
        "a_low": 1.0, "a_high": 2.0, "iters_done": int(done), "delta": [float(delta[0])],
        "index_seed": 7, "index": [int(v) for v in idx], "rank": [int(v) for v in k],
        "gap_over_rms": [float(v) for v in gap],
    }
    with open(os.path.join(HERE, f"one_step_2p{lg}.json"), "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    for lg in ([int(a) for a in sys.argv[1:]] or sorted(CASES)):
        make(lg)
        print(f"wrote one_step_2p{lg}.json", flush=True)
