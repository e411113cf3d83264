"""Threshold and slope of the oracle under each candidate reading.

TEST INFRASTRUCTURE ONLY: calls nothing but the oracle in this folder.

The paper prints p_c ~ 7.3% and a slope gamma ~ 1/5 of
p_log = C (p/p_c)^(gamma L) for the synchronous 2D decoder (Sec. 7.2,
captions of the p_log figures).  The rule's printed form is garbled or
ambiguous in a few places (Def. "message passing automaton, general
dimensions": the line C^{(a)}, the force f^a with an absent message, the
degeneracy-breaking key of eq. (degbreak)).  This script decodes the same
seeded samples under each candidate reading at a fixed budget and reports,
per reading: p_log against p for L = 16, 32, 64, the crossings of
consecutive sizes (timeouts counted as failures, and among terminated
samples only), and gamma from L = 16/32 at p = 5% and 6%.

    python -m oracle.readings_table --n 10000 --json out.json
"""
from __future__ import annotations

import argparse
import json
import math
import time

import numpy as np

from . import oracle as o

READINGS = [
    ("adopted (R1-R5)", 0),
    ("literal sign of f^a", o.READ_LITERAL_SIGN),
    ("literal key m + s a/3", o.READ_LITERAL_KEY),
    ("literal sign and key", o.READ_LITERAL_SIGN | o.READ_LITERAL_KEY),
    ("move on axis ties", o.READ_TIE_MOVES),
    ("mirrored tie order", o.READ_TIE_MIRROR),
    ("C = single site", o.READ_LINE_SITE),
    ("C = unit ball", o.READ_LINE_BALL),
]

PS = [0.05, 0.055, 0.06, 0.065, 0.07, 0.075, 0.08, 0.085, 0.09, 0.095]
SIZES = (16, 32, 64)


def seeds(config_id: int, p_index: int, n: int):
    """(config_id << 40) | (p_index << 32) | i, as the workloads use."""
    return (np.uint64(config_id) << np.uint64(40)) | (np.uint64(p_index) << np.uint64(32)) | np.arange(
        n, dtype=np.uint64)


def crossing(ps, a, b):
    """First p where b - a turns from negative to positive (linear)."""
    d = np.asarray(b) - np.asarray(a)
    for k in range(1, len(ps)):
        if d[k - 1] < 0 <= d[k]:
            return ps[k - 1] + (ps[k] - ps[k - 1]) * (-d[k - 1]) / (d[k] - d[k - 1])
    return None


def gamma(p, pc, pl_small, pl_big, dL):
    if pc is None or pl_small <= 0 or pl_big <= 0:
        return None
    return math.log(pl_big / pl_small) / (dL * math.log(p / pc))


def run(n: int, T_max: int, threads: int, which=None):
    out = []
    for name, bits in READINGS:
        if which is not None and bits not in which:
            continue
        o.set_reading(bits)
        t0 = time.time()
        row = dict(reading=name, bits=bits, n=n, T_max=T_max, p=PS, p_log={}, p_log_done={}, timeouts={},
                   mean_T={})
        for L in SIZES:
            pl, pd, to, mt = [], [], [], []
            for i, p in enumerate(PS):
                r = o.decode_seeds(L, p, seeds(96, 100 * L + i, n), T_max, threads=threads, want_sigma=False)
                fl = r["flags"]
                done = (fl & 2) == 0
                pl.append(float((fl & 1).mean()))
                pd.append(float((fl[done] & 1).mean()) if done.any() else float("nan"))
                to.append(float((~done).mean()))
                mt.append(float(r["T_dec"][done].mean()) if done.any() else float("nan"))
            row["p_log"][L], row["p_log_done"][L], row["timeouts"][L], row["mean_T"][L] = pl, pd, to, mt
        row["crossing"] = {f"{a}/{b}": crossing(PS, row["p_log"][a], row["p_log"][b])
                           for a, b in zip(SIZES, SIZES[1:])}
        row["crossing_done"] = {f"{a}/{b}": crossing(PS, row["p_log_done"][a], row["p_log_done"][b])
                                for a, b in zip(SIZES, SIZES[1:])}
        pc = row["crossing"]["16/32"]
        row["gamma_own_pc"] = [gamma(PS[i], pc, row["p_log"][16][i], row["p_log"][32][i], 16) for i in (0, 2)]
        row["gamma_7.3"] = [gamma(PS[i], 0.073, row["p_log"][16][i], row["p_log"][32][i], 16) for i in (0, 2)]
        row["seconds"] = time.time() - t0
        out.append(row)
        print(json.dumps({k: row[k] for k in ("reading", "crossing", "crossing_done", "gamma_own_pc",
                                               "gamma_7.3", "seconds")}), flush=True)
    o.set_reading(0)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=10000, help="samples per (reading, L, p)")
    ap.add_argument("--T_max", type=int, default=512)
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--bits", type=int, nargs="*", default=None, help="only these readings")
    ap.add_argument("--json", default=None)
    a = ap.parse_args()
    res = run(a.n, a.T_max, a.threads, a.bits)
    if a.json:
        with open(a.json, "w") as f:
            json.dump(res, f, indent=1)


if __name__ == "__main__":
    main()
