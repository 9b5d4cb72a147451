"""Oracle A_H of a 1-in-50 sample of the serving request stream.

Every 50th of the 10,000 seeded requests (hom_inputs.serving_stream with the
bench's geometry pool) is solved by the FP64 oracle (oracle/, naive DFT) at
tol 1e-10 and its A_H written to serving_samples.json, smallest cells first,
one record at a time, so a run that is stopped keeps what it finished.  The
3-D 127^3 requests take tens of minutes each on 8 cores; by default only
--max-127 of them are solved.

    python tests/golden/make_serving_golden.py [--max-127 K]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import hom_inputs as hi  # noqa: E402
from oracle import oracle  # noqa: E402

TOL = 1e-10
PATH = os.path.join(HERE, "serving_samples.json")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--max-127", type=int, default=4)
    a = ap.parse_args()
    reqs = hi.serving_stream(10_000, rate=500.0, seed=5, geometry_pool=16)[::50]
    reqs = sorted(reqs, key=lambda r: (int(np.prod(r.N)), r.idx))
    done = {}
    if os.path.exists(PATH):
        with open(PATH) as fh:
            done = {rec["idx"]: rec for rec in json.load(fh)["requests"]}
    n127 = sum(1 for r in done.values() if r["N"][0] == 127 and r["d"] == 3)
    for r in reqs:
        if r.idx in done:
            continue
        if r.d == 3 and r.N[0] == 127:
            if n127 >= a.max_127:
                continue
            n127 += 1
        t0 = time.time()
        c = oracle.Cell(r.field(), r.N)
        _, W, _, its = c.solve(r.E, tol=TOL)
        done[r.idx] = {"idx": r.idx, "d": r.d, "N": list(r.N), "L": int(r.E.shape[0]),
                       "contrast": r.contrast, "microstructure": r.kind_micro,
                       "W": W.tolist(), "iters": [int(i) for i in its],
                       "seconds": time.time() - t0}
        with open(PATH + ".tmp", "w") as fh:
            json.dump({"source": "tests/golden/make_serving_golden.py: FP64 oracle at tol %g on "
                                 "every 50th request of hom_inputs.serving_stream(10000, seed 5, "
                                 "geometry_pool 16)" % TOL,
                       "tol": TOL, "requests": sorted(done.values(), key=lambda q: q["idx"])},
                      fh, indent=0)
        os.replace(PATH + ".tmp", PATH)
        print(f"request {r.idx} d={r.d} N={r.N[0]} L={r.E.shape[0]} contrast {r.contrast:.0f}: "
              f"{time.time() - t0:.1f} s", flush=True)


if __name__ == "__main__":
    main()
