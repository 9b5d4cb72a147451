"""Write the stored expected values of the full-size parity tests.

Every number here comes from the FP64 oracle (oracle/, naive DFT, the paper's
real-space CG of Sec. 5.3 and the energy quadrature) on the seeded inputs of
hom_inputs; nothing is taken from the GPU path.  The discrete problem has a
unique solution (Sec. 5.2-5.3), so a tight tolerance fixes it to round-off
times the contrast.

    python tests/golden/make_golden.py square    # 15 x 15, seconds
    python tests/golden/make_golden.py pixels    # 1023 x 1023, tens of minutes

square: W and J of E = e1, e2, the iteration count at the configuration
tolerance 1e-8 and the whole strain field; pixels: W and J of E = e1, e2 and
the strain at 64 seeded grid points of each load case.
"""
from __future__ import annotations

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

TOL = 1e-13


def sample_points(N, count, seed):
    """count grid points (index tuples) drawn with the SplitMix64 generator."""
    u = hi.uniform(seed, count * len(N))
    return [[int(u[i * len(N) + a] * N[a]) for a in range(len(N))] for i in range(count)]


def square():
    w = hi.cfg1_square()
    c = oracle.Cell(w.A, w.N)
    E = np.eye(2)
    t0 = time.time()
    x, W, J, its = c.solve(E, tol=TOL)
    _, it8, _ = c.cg(w.E[0], tol=w.tol)
    strain = x + E[:, :, None, None]
    return {"workload": w.name, "N": list(w.N), "E": E.tolist(), "tol": TOL,
            "W": W.tolist(), "J": J.tolist(), "iters": [int(i) for i in its],
            "iters_at_config_tol": {"E": w.E[0].tolist(), "tol": w.tol, "iters": int(it8)},
            "strain": strain.tolist(), "seconds": time.time() - t0}


def pixels():
    w = hi.cfg2_pixels()
    c = oracle.Cell(w.A, w.N)
    E = np.eye(2)
    t0 = time.time()
    x, W, J, its = c.solve(E, tol=TOL)
    pts = sample_points(w.N, 64, seed=1023)
    samples = [[[float(x[l, a][tuple(p)] + E[l, a]) for a in range(2)] for p in pts]
               for l in range(2)]
    return {"workload": w.name, "N": list(w.N), "E": E.tolist(), "tol": TOL,
            "W": W.tolist(), "J": J.tolist(), "iters": [int(i) for i in its],
            "points": pts, "strain_at_points": samples, "seconds": time.time() - t0}


def main():
    which = sys.argv[1:] or ["square"]
    for name in which:
        rec = {"square": square, "pixels": pixels}[name]()
        rec["source"] = ("tests/golden/make_golden.py: FP64 oracle (naive DFT, CG of Sec. 5.3, "
                         "energy quadrature W_lm = <e_l . A e_m>) at tol %g on hom_inputs" % TOL)
        path = os.path.join(HERE, f"{name}.json")
        with open(path, "w") as fh:
            json.dump(rec, fh, indent=1)
        print(f"wrote {path} ({rec['seconds']:.1f} s, iterations {rec['iters']})")


if __name__ == "__main__":
    main()
