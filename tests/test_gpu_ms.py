"""The Moulinec-Suquet scheme on the GPU operator (hom_solve_ms) against the
oracle's Neumann series (Sec. 5.3), and the iteration counts of MS and CG
against the contrast: linear for MS, square root for CG."""
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


@gpu
@pytest.mark.parametrize("N,kind,scheme", [((15, 13), 0, 0), ((9, 7, 11), 1, 0), ((9, 11), 2, 1)])
def test_ms_matches_oracle(hom, oracle, N, kind, scheme):
    """Same steps x <- x + (b - G A x) / lambda on both sides: equal step
    counts (+-1) and fields to round-off at tol 1e-10; at tol 1e-12 the MS
    result is the oracle's CG solution (the unique discrete solution)."""
    d = len(N)
    Q = tuple(2 * n - 1 for n in N) if scheme == 1 else N
    A = hi.random_spd_field(Q, kind, seed=101 + kind, contrast=10.0)
    ocell = oracle.Cell(A, N, kind=kind, scheme=scheme)
    g = hom.Cell(A, N, kind=kind, scheme=scheme)
    E = np.eye(d)[0]
    # lambda from the coefficient's eigenvalue range, as the library takes it
    if kind == 0:
        ev = A.reshape(-1)
    elif kind == 1:
        ev = A.reshape(d, -1).reshape(-1)
    else:
        from test_oracle_pins import _A_matrix_at
        Af = A.reshape(A.shape[0], -1)
        ev = np.concatenate([np.linalg.eigvalsh(_A_matrix_at(Af, kind, d, p))
                             for p in range(Af.shape[1])])
    lam = 0.5 * (ev.min() + ev.max())
    e_ref, it_ref = ocell.ms(E, lam, tol=1e-10, max_iter=100000)
    r = g.solve_ms(E[None], tol=1e-10, want_strain=True)
    assert abs(r["info"]["iters_inner"] - it_ref) <= 1
    assert rel(r["strain"].cpu().numpy()[0], e_ref) < 1e-9
    assert r["info"]["rel_resid_true"] <= 1e-10
    x, W, _, _ = ocell.solve(np.eye(d), tol=1e-13)
    r12 = g.solve_ms(np.eye(d), tol=1e-12, want_strain=True)
    assert rel(r12["W"], W) < 1e-10
    ref = x + np.eye(d).reshape((d, d) + (1,) * d)
    assert rel(r12["strain"].cpu().numpy(), ref) < 1e-10


@gpu
def test_ms_budget(hom):
    N = (15, 15)
    A = hi.bernoulli_majority(N, 0.4, 3, 100.0, 1.0, seed=7)
    g = hom.Cell(A, N, max_iter=5)
    r = g.solve_ms([[1.0, 0.0]], tol=1e-10, allow=(-4,))
    assert r["status"] == -4
    assert r["info"]["iters_inner"] == 5


@gpu
def test_ms_linear_cg_sqrt_in_contrast(hom):
    """Steps to tol 1e-6 on a 63 x 63 pixel cell for rho_A = 10, 100, 1000:
    fitted log-log slope near 1 for MS (rate (rho_A - 1)/(rho_A + 1)), near
    1/2 or below for CG (Sec. 5.3)."""
    N = (63, 63)
    rhos = [10.0, 100.0, 1000.0]
    ms, cg = [], []
    for rho in rhos:
        A = hi.bernoulli_majority(N, 0.4, 3, rho, 1.0, seed=11)
        g = hom.Cell(A, N)
        cg.append(g.solve([[1.0, 0.0]], tol=1e-6)["info"]["iters_inner"])
        ms.append(g.solve_ms([[1.0, 0.0]], tol=1e-6)["info"]["iters_inner"])
        g.close()
    s_ms = np.polyfit(np.log(rhos), np.log(ms), 1)[0]
    s_cg = np.polyfit(np.log(rhos), np.log(cg), 1)[0]
    assert s_ms > 0.8, (ms, s_ms)
    assert s_cg < 0.6, (cg, s_cg)
