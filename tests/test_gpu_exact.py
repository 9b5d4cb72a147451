"""Ga with exact integration for coefficients given by their Fourier
coefficients (the a_trig option): the library takes the M-grid samples of the
truncated series, which may dip below 0 near jumps, and must reproduce the
oracle on the same samples; without the option such samples are rejected as
not positive definite (A2 per point)."""
import numpy as np
import pytest

import hom_inputs as hi

gpu = pytest.mark.gpu


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.fixture(scope="module")
def hom():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1311_0089_amd as h
    h.lib()
    return h


CASES = {
    "laminate": lambda: ((17, 5), hi.laminate_step_trig((17, 5), 0.3, 100.0, 1.0)),
    "square": lambda: ((15, 15), hi.square_inclusion_trig((15, 15), 0.25, 100.0, 1.0)),
    "spheres": lambda: ((9, 11, 7), hi.inclusions_trig((9, 11, 7), 3, 0.12, 50.0, 1.0, seed=3)),
}


@gpu
@pytest.mark.parametrize("name", sorted(CASES))
def test_ga_exact_matches_oracle(hom, oracle, name):
    N, A = CASES[name]()
    d = len(N)
    assert A.min() < 0.0 or name == "spheres"
    ocell = oracle.Cell(A, N, scheme=1)
    x, W, J, _ = ocell.solve(np.eye(d), tol=1e-13)
    g = hom.Cell(A, N, scheme=hom.GA, a_trig=True)
    r = g.solve(np.eye(d), tol=1e-13, want_strain=True)
    assert rel(r["W"], W) < 1e-10
    assert rel(r["strain"].cpu().numpy(), x + np.eye(d).reshape((d, d) + (1,) * d)) < 1e-10
    g32 = hom.Cell(A, N, scheme=hom.GA, prec=hom.MIXED, a_trig=True)
    assert rel(g32.solve(np.eye(d), tol=1e-7)["W"], W) < 1e-6
    if A.min() <= 0.0:
        with pytest.raises(hom.HomError) as ei:
            hom.Cell(A, N, scheme=hom.GA)
        assert ei.value.code == -2
        assert r["info"]["rho_A"] == float("inf")
    with pytest.raises(hom.HomError):          # only with the doubled grid
        hom.Cell(np.ones(N), N, a_trig=True)
