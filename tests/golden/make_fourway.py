"""Writes fourway_oracle.json: the FP64 oracle's ST-HOSVD of the 4-way field.

Workload: 13 independent 200 x 500 x 500 float32 fields (seeds 100..112)
stacked on the last mode, relative error 1e-3, default mode order (increasing
length: 3, 0, 1, 2), adaptive rank rule.  Recorded per mode: the oracle's
rank, discarded energy, budget share and the full descending eigenvalue list
(so that a boundary-degenerate rank can be judged against the oracle's own
tails), plus |A|^2 and the predicted SSE.  Calls only the oracle and the input
generator.

Run from the repository root:  python tests/golden/make_fourway.py
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

EPS = 1e-3


def main():
    t0 = time.time()
    x = synth.field4()
    t1 = time.time()
    t = oracle.sthosvd(x, EPS)
    t2 = time.time()
    rec = {
        "workload": "13 x F((200, 500, 500), seed 100 + f) stacked on the last mode, float32",
        "shape": list(x.shape),
        "eps": EPS,
        "order": t.order,
        "ranks": t.ranks,
        "norm2": t.norm2,
        "sse_pred": t.sse_pred,
        "tails": t.tails,
        "budgets": t.budgets,
        "eigvals": [[float(v) for v in lam] for lam in t.eigvals],
        "oracle_seconds": round(t2 - t1, 1),
    }
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fourway_oracle.json")
    with open(out, "w") as f:
        json.dump(rec, f, indent=1)
    print("generated in %.1f s, oracle %.1f s, ranks %s -> %s" % (t1 - t0, t2 - t1, t.ranks, out))


if __name__ == "__main__":
    main()
