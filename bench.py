"""Benchmark: dense generalized symmetric-definite eigenproblems on one MI355X.

One step = one full FP64 solve (all eigenpairs) of the M = 32768 workload
(decay length 64, seed 3) through gep_solve: Cholesky, reduced matrix, full ->
band -> tridiagonal, divide and conquer, both back transformations and
Y = L^{-T} Z.  Inputs are resident in HBM before the timed region.

Prints one JSON line (see the repository's design notes for the field meanings).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "GEP solves/s + FP64 TFLOP/s at M=32768; mixed-vs-FP64 speedup at 1e-11 err"
PEAK_FP64 = 78.6  # TFLOP/s, MI355X dense FP64 (matrix == vector)
PHASE_FLOPS = {
    # algorithmic flops per phase, M^3 coefficients (band width b enters S2 only)
    "R1": lambda M, b: M ** 3 / 3.0,
    "R2-4": lambda M, b: M ** 3 * 1.0,
    "S1": lambda M, b: 4.0 * M ** 3 / 3.0,
    "S2": lambda M, b: 6.0 * b * M ** 2,
    "S4": lambda M, b: 2.0 * M ** 3,
    "S5": lambda M, b: 2.0 * M ** 3,
    "R5": lambda M, b: M ** 3 * 1.0,
}


def band_width(M: int) -> int:
    return 64 if M >= 2048 else (32 if M >= 256 else 16)


def alg_flops(M: int) -> float:
    """(23/3) M^3 + 6 b M^2: every phase except the divide and conquer, whose
    deflation-dependent flops are not counted."""
    b = band_width(M)
    return sum(f(M, b) for f in PHASE_FLOPS.values())


def cpu_baseline(M_target: int, sample: int) -> dict:
    """The CPU oracle (plain C, OpenMP) on a bounded sample: one full solve of the
    same generator at order `sample`, scaled to order M_target by (M/sample)^3."""
    import oracle
    import synth
    A, B = synth.banded_pair(sample, synth.decay_length(sample), 3)
    oracle.lib()
    t0 = time.perf_counter()
    r = oracle.solve(A, B)
    dt = time.perf_counter() - t0
    assert r.info == 0
    scale = (M_target / sample) ** 3
    return {"value": 1.0 / (dt * scale), "unit": "solves/s", "cores": oracle.threads(),
            "kind": "oracle",
            "sample": f"one full FP64 oracle solve at M={sample} ({dt:.2f} s), scaled by "
                      f"(M/{sample})^3 to M={M_target}"}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--size", type=int, default=32768)
    ap.add_argument("--cpu-sample", type=int, default=1536)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this solver runs on one GPU; multi-GPU runs are not supported "
              f"(asked for --gpus {args.gpus})", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import synth
    import paper_1504_06443_amd as gep

    M = args.size
    ell = synth.decay_length(M) if M != 32768 else 64.0
    seed = 3 if M == 32768 else 2
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    A, B = synth.banded_pair(M, ell, seed)
    print(f"[bench] generated M={M} in {time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)
    dA = torch.from_numpy(A).to(dev)
    dB = torch.from_numpy(B).to(dev)
    del A, B
    torch.cuda.synchronize()

    gep.profile_enable(True)
    for i in range(args.warmup):
        lam, Y = gep.solve(dA, dB)
        torch.cuda.synchronize()
        print(f"[bench] warmup {i} done", file=sys.stderr, flush=True)
        del lam, Y
    times = []
    phases = {}
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.steps):
        ts = time.perf_counter()
        lam, Y = gep.solve(dA, dB, check_info=False)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - ts)
        ph = gep.profile_read()
        for k, v in ph.items():
            phases.setdefault(k, []).append(v)
        print(f"[bench] step {i}: {times[-1]:.3f}s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ms_per_step = 1000.0 * elapsed / args.steps
    solves_per_s = args.steps / elapsed
    F = alg_flops(M)
    tflops = F / (elapsed / args.steps) / 1e12
    phase_ms = {k: float(np.median(v)) for k, v in phases.items()}

    # dominant phase and its roofline (MFMA-bound phases against the FP64 peak)
    b = band_width(M)
    dom = max((k for k in phase_ms if k in PHASE_FLOPS), key=lambda k: phase_ms[k])
    dom_tf = PHASE_FLOPS[dom](M, b) / (phase_ms[dom] / 1e3) / 1e12
    bound = "alu" if dom == "S2" else "mfma"
    roofline = {"bound": bound, "achieved": dom_tf, "peak": PEAK_FP64, "unit": "TFLOP/s",
                "frac": dom_tf / PEAK_FP64, "traffic": None, "phase": dom,
                "phase_ms": phase_ms[dom]}

    check = None
    if not args.no_check:
        info = gep.api._info(dev)
        # invariants at full size, on the GPU with torch matmuls (independent of libgep)
        with torch.no_grad():
            Asym = torch.triu(dA) + torch.triu(dA, 1).t()
            Bsym = torch.triu(dB) + torch.triu(dB, 1).t()
            Yc = Y.contiguous()
            AY = Asym @ Yc
            BY = Bsym @ Yc
            n1 = Asym.abs().sum(0).max().item()
            res = ((AY - BY * lam[None, :]).abs().sum(0).max() / (n1 * Yc.abs().sum(0).max())).item()
            del AY
            G = Yc.t() @ BY
            G.diagonal().sub_(1.0)
            orth = G.abs().max().item()
            del G, BY
        check = {"residual": res, "orth": orth, "norm1_A": n1}

    out = {
        "metric": METRIC,
        "value": solves_per_s,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"gep_fp64_m{M}_decay{ell:g}_seed{seed}", "M": M,
                   "band_width": b, "job": "vectors", "precision": "fp64"},
        "tflops_fp64": tflops,
        "alg_flops_per_solve": F,
        "phase_ms": phase_ms,
        "mixed_speedup": None,
        "roofline": roofline,
        "check": check,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(M, args.cpu_sample)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
