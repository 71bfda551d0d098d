"""Write paper_2011_11120_amd/data/kappa.json: the scale of the synthetic reflection kernels.

The Marchenko operator M = [[I, -Theta R], [-Theta R*, I]] (Eq.5) is well
conditioned when every slice has ||K_f||_2 <= q < 1 (sigma(M) in [1-q, 1+q]).
For the 2500-trace workload the spectral norm of sampled slices is taken with
the FP64 oracle's power iteration on host-generated slices; for the
10000-trace workload (too large to generate on the host) the Frobenius norm
of sampled rows bounds the spectral norm from above.  Only the seeded input
generator and oracle.power are used.  The value is an input parameter of the
workload generators, so it is stored as package data, not as a test fixture.

    python tests/golden/make_kappa.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import power  # noqa: E402
from paper_2011_11120_amd import synth, workloads  # noqa: E402

TARGET = 0.5


def c4():
    spec = workloads.marchenko_spec(nx=50, nt=1024, nfmax=250)
    bins = [10, 25, 40, 50, 61, 70, 85, 100, 130, 170, 220]
    idx = np.arange(spec.n)
    norms, ratio = {}, 0.0
    for f in bins:
        K = synth.kernel_block(spec, [f], idx, idx)[0]
        norms[f] = power.spectral_norm(K, iters=60)
        ratio = max(ratio, norms[f] / float(np.linalg.norm(K)))
        print(f"c4 bin {f}: ||K_f||_2 = {norms[f]:.4e}", flush=True)
    return {"kappa": TARGET / max(norms.values()), "target": TARGET, "method": "power iteration, sampled bins",
            "bins": bins, "norms": [norms[f] for f in bins], "spectral_over_frobenius_max": ratio}


def c5(ratio):
    spec = workloads.marchenko_spec(nx=100, nt=1024, nfmax=200)
    rng = np.random.default_rng(0)
    rows = np.sort(rng.choice(spec.n, 40, replace=False))
    bins = [10, 25, 40, 50, 61, 70, 85, 100, 130, 170]
    idx = np.arange(spec.n)
    fro = {}
    for f in bins:
        K = synth.kernel_block(spec, [f], rows, idx)[0]
        fro[f] = float(np.sqrt(np.sum(np.abs(K) ** 2) * spec.n / rows.size))
        print(f"c5 bin {f}: ||K_f||_F ~ {fro[f]:.4e}", flush=True)
    return {"kappa": TARGET / (ratio * max(fro.values())), "target": TARGET,
            "method": "Frobenius norm from 40 sampled rows times the spectral/Frobenius ratio of the 2500-trace slices",
            "bins": bins, "norms": [fro[f] for f in bins], "ratio": ratio}


if __name__ == "__main__":
    a = c4()
    out = {"c4": a, "c5": c5(a["spectral_over_frobenius_max"])}
    dst = os.path.join(os.path.dirname(os.path.dirname(HERE)), "paper_2011_11120_amd", "data", "kappa.json")
    with open(dst, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps({k: v["kappa"] for k, v in out.items()}))
