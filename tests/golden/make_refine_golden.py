"""Write refine_grad_fd.json: central finite differences of the FP64 oracle
for the gradient of 2F at one bin, on the refinement workload at full size
(2 detectors x 30 d at 1 s, n_fft 2^22, 0.2 Hz band at 400 Hz).

Calls only oracle/ (and the seeded input generator).  For each of four
candidates (one per injection 0-3) and each of the five parameters the
refinement moves (df, f1dot, asini, porb, tp), the derivative of
L = 2F(bin) is (L(x + h) - L(x - h)) / 2h with h a thousandth of the
parameter's metric scale, and again with 2h (the two agree to the
truncation error, which is reported).  Run: python tests/golden/make_refine_golden.py
"""
import json
import math
import os
import sys
from concurrent.futures import ProcessPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

CANDIDATES = (0, 9, 18, 27)
PARAMS = ("df", "f1dot", "asini", "porb", "tp")
COL = {"df": 2, "f1dot": 3, "asini": 5, "porb": 6, "tp": 7}

_DS = None


def dataset():
    global _DS
    if _DS is None:
        from paper_2201_00451_amd import synth
        _DS = synth.config_refine()
    return _DS


def scales(ds, m):
    inj = ds.injections[ds.cand_inj[m]]
    T = ds.detectors[0].n * ds.dt
    om = 2.0 * math.pi / inj["porb"]
    f, a = inj["f"], inj["asini"]
    return {"df": 1.0 / T, "f1dot": 1.0 / T ** 2, "asini": 1.0 / (2 * math.pi * f),
            "porb": inj["porb"] ** 2 / (2 * math.pi * f * a * T),
            "tp": 1.0 / (2 * math.pi * f * a * om)}


def value(args):
    m, name, delta = args
    from oracle import fstat_oracle as O
    ds = dataset()
    row = ds.templates[m].copy()
    if name is not None:
        row[COL[name]] += delta
    return O.twoF_at_bin(ds, row, int(ds.cand_bins[m]))


def main():
    ds = dataset()
    jobs = []
    for m in CANDIDATES:
        jobs.append((m, None, 0.0))
        sc = scales(ds, m)
        for name in PARAMS:
            h = 1e-3 * sc[name]
            for d in (h, -h, 2 * h, -2 * h):
                jobs.append((m, name, d))
    with ProcessPoolExecutor(max_workers=4) as ex:
        vals = list(ex.map(value, jobs))
    res = dict(zip([(m, n, d) for m, n, d in jobs], vals))
    out = {"workload": "refinement workload (synth.config_refine defaults): 2 detectors x "
                       "2592000 samples, n_fft 2^22, 0.2 Hz band at 400 Hz",
           "method": "central differences of the FP64 oracle's 2F at the candidate's bin "
                     "(oracle.fstat_oracle.twoF_at_bin), step h = 1e-3 metric scale; "
                     "grad_2h uses 2h",
           "candidates": []}
    for m in CANDIDATES:
        sc = scales(ds, m)
        ent = {"index": m, "bin": int(ds.cand_bins[m]), "twoF": res[(m, None, 0.0)],
               "grad": {}, "grad_2h": {}, "step": {}}
        for name in PARAMS:
            h = 1e-3 * sc[name]
            ent["step"][name] = h
            ent["grad"][name] = (res[(m, name, h)] - res[(m, name, -h)]) / (2 * h)
            ent["grad_2h"][name] = (res[(m, name, 2 * h)] - res[(m, name, -2 * h)]) / (4 * h)
        out["candidates"].append(ent)
        print(json.dumps(ent), flush=True)
    with open(os.path.join(HERE, "refine_grad_fd.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
