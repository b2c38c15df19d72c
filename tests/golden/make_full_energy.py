"""Write the FP64 oracle's total potential energy U and virial W of the
jittered N = 256,000 workload (40^3 FCC at rho = 0.8442, jitter 0.05 sigma
with the workload's seed) to ``lj256k_jitter_energy.json``.

The O(N^2) brute-force sum takes about a minute on 8 host cores, too long
for every test run, so its result is stored once. This script calls only the
oracle and the seeded input generator; rerun it to regenerate the file:

    python tests/golden/make_full_energy.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import ljsynth  # noqa: E402
import oracle  # noqa: E402

OUT = os.path.join(HERE, "lj256k_jitter_energy.json")
JITTER = 0.05


def main():
    oracle.build(force=False)
    w = ljsynth.WORKLOADS["lj256k"]
    pos4, _, box = ljsynth.make_state(w, jitter_amp=JITTER)
    p = oracle.params(box)
    rows = np.arange(w.n)
    u = w_sum = 0.0
    for r0 in range(0, w.n, 16384):  # rows in chunks; the per-row halves sum to the totals
        _, ur, wr = oracle.forces_rows(p, pos4, rows[r0:r0 + 16384])
        u += float(ur.sum())
        w_sum += float(wr.sum())
        print(f"rows {r0 + len(ur)} / {w.n}", flush=True)
    rec = {
        "source": "FP64 brute-force oracle (oracle/lj_oracle.c) over all N^2 ordered pairs, written by "
                  "tests/golden/make_full_energy.py",
        "workload": w.name, "n": w.n, "density": w.density, "jitter": JITTER, "seed": w.seed,
        "box": box, "U": u, "W": w_sum,
    }
    with open(OUT, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
