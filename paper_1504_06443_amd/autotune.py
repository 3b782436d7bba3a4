"""Autotuner: times gep_solve on the GPU for candidate values of the tunable
parameters over ranges of orders and writes the fastest into tuning.json beside
libgep.so, which the library reads when it is first used (include/gep.h,
"Tuned parameters").

    python -m paper_1504_06443_amd.autotune [--out PATH] [--quick]

For each range of orders a representative order (the geometric middle) is
solved with the synthetic Hamiltonian / overlap generator (decay length
sqrt(M/8)); every candidate is timed as the median of several solves after a
warm-up, and the winner must beat the built-in rule by more than 2% to replace
it.  Parameters are tuned one after another (band width, then the
divide-and-conquer leaf with the chosen band width), and the Q2 kernel choice is
timed on its own phase at the large orders.  The file records every timing, so
the table's effect can be read from it.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# (m_lo, m_hi) ranges of orders for band width and leaf size
RANGES = [(64, 127), (128, 255), (256, 511), (512, 1023), (1024, 2047), (2048, 4095),
          (4096, 8191)]
BAND_CANDIDATES = (8, 16, 24, 32, 48, 64)
LEAF_CANDIDATES = (16, 32, 48, 64)
MARGIN = 0.02


def _rep(lo: int, hi: int) -> int:
    return max(lo, min(hi, int(round(math.sqrt(lo * (hi + 1))))))


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(HERE, "tuning.json"))
    ap.add_argument("--quick", action="store_true", help="fewer repetitions")
    ap.add_argument("--max-order", type=int, default=8191)
    args = ap.parse_args()

    import torch
    import synth
    from paper_1504_06443_amd import _binding
    import paper_1504_06443_amd as gep

    L = _binding.lib()
    L.gep_tune_clear()  # time against the built-in rules, not an older table

    def timed(dA, dB, reps):
        gep.solve(dA, dB, check_info=False)
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            gep.solve(dA, dB, check_info=False)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        return sorted(ts)[len(ts) // 2] * 1e3

    def sweep(key, M, candidates, reps, dA, dB):
        res = {}
        for v in candidates:
            L.gep_tune_reset_overrides()
            for k, val in fixed.items():
                L.gep_tune_set(k.encode(), M, M, val)
            assert L.gep_tune_set(key.encode(), M, M, v) == 0
            res[v] = timed(dA, dB, reps)
            print(f"[autotune] {key} M={M} value={v}: {res[v]:.3f} ms", flush=True)
        L.gep_tune_reset_overrides()
        return res

    params = {"band_width": [], "dc_leaf": [], "q2_wide_min_cols": []}
    log = []
    for lo, hi in RANGES:
        if lo > args.max_order:
            break
        M = _rep(lo, hi)
        reps = 3 if (args.quick or M >= 2048) else 7
        A, B = synth.banded_pair(M, synth.decay_length(M), 31000 + M)
        dA = torch.from_numpy(A).cuda()
        dB = torch.from_numpy(B).cuda()
        fixed = {}
        b_default = int(L.gep_tune_get(b"band_width", M))
        cands = sorted({b for b in BAND_CANDIDATES if b < M} | {b_default})
        tb = sweep("band_width", M, cands, reps, dA, dB)
        best_b = min(tb, key=tb.get)
        if tb[best_b] > (1.0 - MARGIN) * tb[b_default]:
            best_b = b_default
        fixed["band_width"] = best_b
        leaf_default = int(L.gep_tune_get(b"dc_leaf", M))
        tl = sweep("dc_leaf", M, sorted({v for v in LEAF_CANDIDATES if v <= max(M, 16)}
                                        | {leaf_default}), reps, dA, dB)
        best_l = min(tl, key=tl.get)
        if tl[best_l] > (1.0 - MARGIN) * tl[leaf_default]:
            best_l = leaf_default
        entry = {"m_lo": lo, "m_hi": hi, "order_timed": M}
        params["band_width"].append(dict(entry, value=best_b,
                                         ms_builtin=tb[b_default], ms_tuned=tb[best_b]))
        params["dc_leaf"].append(dict(entry, value=best_l, ms_builtin=tl[leaf_default],
                                      ms_tuned=tl[best_l]))
        log.append({"M": M, "band_width_ms": tb, "dc_leaf_ms": tl})
        del dA, dB
        torch.cuda.empty_cache()

    # Q2 back transformation: 16 or 32 columns per wave, on its own phase time
    for M in (8192, 16384, 32768):
        if M > 4 * args.max_order + 4:
            break
        A, B = synth.banded_pair(M, synth.decay_length(M), 32000 + M)
        dA = torch.from_numpy(A).cuda()
        dB = torch.from_numpy(B).cuda()
        del A, B
        gep.profile_enable(True)
        q2 = {}
        for label, thr in (("16_per_wave", M + 1), ("32_per_wave", 0)):
            L.gep_tune_reset_overrides()
            L.gep_tune_set(b"q2_wide_min_cols", M, M, thr)
            gep.solve(dA, dB, check_info=False)
            torch.cuda.synchronize()
            ph = []
            for _ in range(1 if M >= 16384 else 3):
                gep.solve(dA, dB, check_info=False)
                torch.cuda.synchronize()
                ph.append(gep.profile_read()["S4"])
            q2[label] = sorted(ph)[len(ph) // 2]
            print(f"[autotune] Q2 M={M} {label}: {q2[label]:.1f} ms", flush=True)
        L.gep_tune_reset_overrides()
        builtin = "32_per_wave" if M >= int(L.gep_tune_get(b"q2_wide_min_cols", M)) else "16_per_wave"
        other = "16_per_wave" if builtin == "32_per_wave" else "32_per_wave"
        best = other if q2[other] < (1.0 - MARGIN) * q2[builtin] else builtin
        params["q2_wide_min_cols"].append(
            {"m_lo": M, "m_hi": 2 * M - 1 if M < 32768 else 1 << 40, "order_timed": M,
             "value": 0 if best == "32_per_wave" else 1 << 40, "ms_builtin": q2[builtin],
             "ms_tuned": q2[best], "phase": "S4"})
        log.append({"M": M, "q2_phase_ms": q2})
        del dA, dB
        torch.cuda.empty_cache()

    out = {"device": torch.cuda.get_device_name(0), "generated": time.strftime("%Y-%m-%d %H:%M:%S"),
           "rule": f"median solve time; the built-in rule is kept unless beaten by >{MARGIN:.0%}",
           "parameters": {k: v for k, v in params.items() if v}, "timings": log}
    with open(args.out, "w") as f:
        json.dump(out, f, indent=1)
    print(f"[autotune] wrote {args.out}", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
