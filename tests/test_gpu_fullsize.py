"""GPU parity at the configuration sizes.

Stored oracle results (tests/golden/*.json, written by make_golden.py from
the FP64 oracle only): the 15 x 15 square inclusion and the 1023 x 1023
pixel microstructure; the discrete solution is unique (Sec. 5.2-5.3), so the
FP64 path must reproduce them to 1e-10 when both sides solve to tol 1e-13
(field errors scale like contrast x tol) and the mixed path's A_H to 1e-6.
Closed forms at the 3-D sizes, where the oracle would need hours: an
isotropic laminate a(x_1) I on 255^3 (GaNi: harmonic mean across the layers,
arithmetic mean along them) and a laminate sampled on the doubled 253^3 grid
of a 127^3 trial space (Ga: the along-layer entries are the arithmetic mean
of the samples exactly, the across-layer entry lies above their harmonic
mean)."""
import json
import os

import numpy as np
import pytest

import hom_inputs as hi

gpu = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def load(name):
    path = os.path.join(GOLDEN, f"{name}.json")
    if not os.path.exists(path):
        pytest.skip(f"{path} not written")
    with open(path) as fh:
        return json.load(fh)


@pytest.fixture(scope="module")
def hom():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1311_0089_amd as h
    h.lib()
    return h


@gpu
def test_square_15_against_stored_oracle(hom):
    g = load("square")
    w = hi.cfg1_square()
    E = np.array(g["E"])
    c64 = hom.Cell(w.A, w.N)
    r = c64.solve(E, tol=g["tol"], want_strain=True)
    assert rel(r["W"], g["W"]) < 1e-10
    assert rel(r["J"], g["J"]) < 1e-10
    assert rel(r["strain"].cpu().numpy(), g["strain"]) < 1e-10
    # at the configuration tolerance the iteration count is the oracle's
    cfg = g["iters_at_config_tol"]
    r8 = c64.solve(np.array([cfg["E"]]), tol=cfg["tol"])
    assert abs(r8["info"]["iters_inner"] - cfg["iters"]) <= 1
    c32 = hom.Cell(w.A, w.N, prec=hom.MIXED)
    r32 = c32.solve(E, tol=1e-6)
    assert rel(r32["W"], g["W"]) < 1e-6


@gpu
def test_pixels_1023_against_stored_oracle(hom):
    g = load("pixels")
    w = hi.cfg2_pixels()
    E = np.array(g["E"])
    c64 = hom.Cell(w.A, w.N)
    r = c64.solve(E, tol=g["tol"], want_strain=True)
    assert rel(r["W"], g["W"]) < 1e-10
    assert rel(r["J"], g["J"]) < 1e-10
    s = r["strain"].cpu().numpy()
    got = [[[s[l, a][tuple(p)] for a in range(2)] for p in g["points"]] for l in range(2)]
    assert rel(got, g["strain_at_points"]) < 1e-10
    # the mixed path at the configuration tolerance
    c32 = hom.Cell(w.A, w.N, prec=hom.MIXED)
    r32 = c32.solve(E, tol=w.tol)
    assert rel(r32["W"], g["W"]) < 1e-6


@gpu
@pytest.mark.parametrize("prec_name", ["FP64", "MIXED"])
def test_laminate_255_cubed_closed_form(hom, prec_name):
    """Isotropic laminate a(x_1) I, 255^3, three load cases batched:
    A_H = diag(harmonic, arithmetic, arithmetic) of the layer values."""
    prec = getattr(hom, prec_name)
    N = (255, 255, 255)
    a = 1.0 + 99.0 * hi.uniform(255, N[0])
    A = hi.laminate(N, a)
    c = hom.Cell(A, N, prec=prec)
    tol = 1e-12 if prec == hom.FP64 else 1e-6
    r = c.solve(np.eye(3), tol=tol)
    ref = np.diag([1.0 / np.mean(1.0 / a), np.mean(a), np.mean(a)])
    bar = 1e-10 if prec == hom.FP64 else 1e-6
    assert np.abs(r["W"] - ref).max() / ref.max() < bar, (prec_name, r["W"])
    c.close()


@gpu
@pytest.mark.parametrize("prec_name", ["FP64", "MIXED"])
def test_ga_laminate_127_on_253_cubed(hom, prec_name):
    """Ga, trial 127^3, laminate sampled on the doubled 253^3 grid: along-layer
    entries equal the arithmetic mean of the samples, the across-layer entry
    is at least their harmonic mean, off-diagonals vanish."""
    prec = getattr(hom, prec_name)
    N = (127, 127, 127)
    M = tuple(2 * n - 1 for n in N)
    a = 1.0 + 30.0 * hi.uniform(253, M[0])
    c = hom.Cell(hi.laminate(M, a), N, scheme=hom.GA, prec=prec)
    tol = 1e-12 if prec == hom.FP64 else 1e-6
    r = c.solve(np.eye(3), tol=tol)
    W = r["W"]
    bar = 1e-10 if prec == hom.FP64 else 1e-6
    assert abs(W[1, 1] - a.mean()) / a.mean() < bar
    assert abs(W[2, 2] - a.mean()) / a.mean() < bar
    assert W[0, 0] >= 1.0 / np.mean(1.0 / a) * (1 - bar)
    off = W - np.diag(np.diag(W))
    assert np.abs(off).max() < bar * a.mean()
    c.close()
