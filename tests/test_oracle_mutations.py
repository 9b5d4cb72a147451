"""Planted mistakes in the oracle must each fail a pin.

Each mutation is one plausible slip in oracle/hom_oracle.c (a dropped term, a
wrong sign or index, a transposed operand); a copy of the source with that
slip is compiled on the CPU and the pin suite runs against it in a
subprocess (the binding loads HOM_ORACLE_LIB).  A mutant on which every pin
still passes would mean the pins do not fix that part of the oracle."""
import concurrent.futures as cf
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "hom_oracle.c")

# (name, text in the source, replacement)
MUTATIONS = [
    ("forward DFT without 1/n", "const double scale = (sign < 0) ? 1.0 / (double)len : 1.0;",
     "const double scale = 1.0;"),
    ("DFT sign flipped", "cs[2 * t + 1] = (double)sign * sin(th);",
     "cs[2 * t + 1] = -(double)sign * sin(th);"),
    ("zero mode kept", "if (k != 0) zero = 0;\n            xi[a] = (double)k / Y[a];\n        }\n        if (zero) {\n            for (int a = 0;",
     "zero = 0;\n            xi[a] = (double)k / Y[a];\n        }\n        if (zero) {\n            for (int a = 0;"),
    ("xi without Y", "xi[a] = (double)k / Y[a];\n        }\n        if (zero) {\n            for (int a = 0;",
     "xi[a] = (double)k;\n        }\n        if (zero) {\n            for (int a = 0;"),
    ("elastic zero mode kept", "if (k != 0) zero = 0;\n            xi[a] = (double)k / Y[a];\n        }\n        if (zero) {\n            for (int q = 0;",
     "zero = 0;\n            xi[a] = (double)k / Y[a];\n        }\n        if (zero) {\n            for (int q = 0;"),
    ("elastic xi without Y", "xi[a] = (double)k / Y[a];\n        }\n        if (zero) {\n            for (int q = 0;",
     "xi[a] = (double)k;\n        }\n        if (zero) {\n            for (int q = 0;"),
    ("projection on the real part only", "z[2 * ((long)a * np + p) + 1] = xi[a] * si / xx;",
     "z[2 * ((long)a * np + p) + 1] = xi[a] * sr / xx;"),
    ("signed index off by one", "static long kof(long i, long n) { return (i <= (n - 1) / 2) ? i : i - n; }",
     "static long kof(long i, long n) { return (i < (n - 1) / 2) ? i : i - n; }"),
    ("flux with a transposed Voigt entry", "s += A_entry(c, np, p, a, b) * e[(long)b * np + p];",
     "s += A_entry(c, np, p, a, a) * e[(long)b * np + p];"),
    ("pad to the wrong position", "q += pos(kof(idx[a], N[a]), M[a]) * stride;\n            stride *= M[a];\n        }\n        for (int c = 0; c < nc; ++c) {\n            zout[2 * ((long)c * nM + q)]",
     "q += idx[a] * stride;\n            stride *= M[a];\n        }\n        for (int c = 0; c < nc; ++c) {\n            zout[2 * ((long)c * nM + q)]"),
    ("RHS sign", "for (long i = 0; i < n; ++i) b[i] = -b[i];", "for (long i = 0; i < n; ++i) b[i] = b[i];"),
    ("beta from the old residual twice", "double beta = rho1 / rho;", "double beta = rho / rho1;"),
    ("alpha without (p, q)", "double alpha = rho / gam;", "double alpha = rho / gdot(n, np, p, p);"),
    ("warm start not re-projected", "else { s = hor_apply_G(c, x, t); memcpy(x, t, sizeof(double) * (size_t)n); free(t); }",
     "else { free(t); }"),
    ("stopping test relative to the warm residual", "double rho0 = (ref2 > 0.0) ? ref2 : rho;",
     "double rho0 = rho;"),
    ("strain without E", "for (long p = 0; p < nQ; ++p) out[(long)a * nQ + p] += E[a];",
     "for (long p = 0; p < nQ; ++p) out[(long)a * nQ + p] += 0.0;"),
    ("W with the strain twice", "W[l * L + m] = gdot((long)nc * nQ, nQ, e + (long)l * nc * nQ, j + (long)m * nc * nQ);",
     "W[l * L + m] = gdot((long)nc * nQ, nQ, e + (long)l * nc * nQ, e + (long)m * nc * nQ);"),
    ("grid mean without 1/|N|", "return s / (double)np;   /* grid mean, Sec. 5.1 */", "return s;"),
    ("elastic projection without the xi xi / (2 |xi|^2) term",
     "ur[a] = (2.0 / xx) * (tr[a] - xi[a] * xtr / (2.0 * xx));", "ur[a] = (2.0 / xx) * tr[a];"),
    ("Mandel shear written without sqrt 2", "double f = (a == b) ? 1.0 : r2;", "double f = 1.0;"),
    ("Hooke law without the trace term", "+ ((q < d) ? lam * tr : 0.0);", "+ 0.0;"),
    ("Hooke law with mu for 2 mu", "j[(long)q * np + p] = 2.0 * mu * e[", "j[(long)q * np + p] = mu * e["),
    ("elastic trace over every component", "for (int a = 0; a < d; ++a) tr += e[(long)a * np + p];",
     "for (int a = 0; a < d * (d + 1) / 2; ++a) tr += e[(long)a * np + p];"),
]


def _run(name, old, new, tmp):
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation target not found: {name}"
    mutant = src.replace(old, new, 1)
    base = os.path.join(tmp, f"m{abs(hash(name)) % 10**8}")
    with open(base + ".c", "w") as fh:
        fh.write(mutant)
    subprocess.check_call(["gcc", "-O1", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                           "-D_DEFAULT_SOURCE", "-I", os.path.join(ROOT, "oracle"), "-o",
                           base + ".so", base + ".c", "-lm"])
    env = dict(os.environ, HOM_ORACLE_LIB=base + ".so", OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    return name, r.returncode


def test_every_planted_mistake_fails_a_pin():
    # the unchanged source, built and run the same way, passes every pin (so a
    # failing mutant fails a pin, not the harness)
    control = ("unchanged", "#include \"hom_oracle.h\"", "#include \"hom_oracle.h\"")
    with tempfile.TemporaryDirectory() as tmp:
        with cf.ThreadPoolExecutor(max_workers=4) as ex:
            results = list(ex.map(lambda m: _run(*m, tmp), [control] + MUTATIONS))
    assert results[0][1] == 0, "the unchanged oracle fails its pins in this harness"
    survivors = [name for name, rc in results[1:] if rc == 0]
    assert not survivors, f"mutants every pin accepts: {survivors}"
