"""Linear elasticity on the GPU (kind ELASTIC, the extension beyond the
scalar setting named in Sec. 6): parity with the oracle's elastic problem
(operator, projection onto compatible strains, solution, effective
stiffness) in 2-D (plane strain) and 3-D, GaNi and Ga, both precisions; the
layered-medium closed form at sizes the oracle cannot reach."""
import numpy as np
import pytest

import hom_inputs as hi
from elastic_ref import elastic_laminate_W, lame_field, lame_stiffness

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
@pytest.mark.parametrize("N,scheme", [((15, 13), 0), ((9, 11), 1), ((33, 31), 0), ((9, 7, 5), 0),
                                      ((7, 5, 9), 1), ((15, 13, 11), 0), ((15, 255), 0),
                                      ((9, 7, 255), 0), ((255, 5, 7), 0)])
def test_elastic_matches_oracle(hom, oracle, N, scheme):
    import torch
    d = len(N)
    m = d * (d + 1) // 2
    Q = tuple(2 * n - 1 for n in N) if scheme == 1 else N
    A = lame_field(Q, 91 + scheme, contrast=30.0)
    oc = oracle.Cell(A, N, kind=oracle.ELASTIC, scheme=scheme)
    x, W, J, _ = oc.solve(np.eye(m), tol=1e-13)
    g = hom.Cell(A, N, kind=hom.ELASTIC, scheme=scheme)
    r = g.solve(np.eye(m), tol=1e-13, want_strain=True)
    assert rel(r["W"], W) < 1e-10
    assert rel(r["J"], J) < 1e-10
    E = np.eye(m).reshape((m, m) + (1,) * d)
    assert rel(r["strain"].cpu().numpy(), x + E) < 1e-10
    mx = hom.Cell(A, N, kind=hom.ELASTIC, scheme=scheme, prec=hom.MIXED)
    assert rel(mx.solve(np.eye(m), tol=1e-8)["W"], W) < 1e-6
    # the operator G C G and the projection onto compatible strains
    u = np.stack([oc.apply_G(hi.normal(160 + l, m * int(np.prod(N))).reshape((m,) + N))
                  for l in range(2)])
    ref = np.stack([oc.apply_GA(u[l]) for l in range(2)])
    assert rel(g.apply(torch.from_numpy(u).cuda()).cpu().numpy(), ref) < 1e-13
    assert rel(g.apply(torch.from_numpy(u).cuda(), hom.MIXED).cpu().numpy(), ref) < 1e-5
    v = hi.normal(170, m * int(np.prod(N))).reshape((1, m) + N)
    assert rel(g.project(torch.from_numpy(v).cuda()).cpu().numpy()[0], oc.apply_G(v[0])) < 1e-13


@gpu
@pytest.mark.parametrize("N", [(255, 63), (63, 31, 15), (255, 127, 63)])
def test_elastic_laminate_closed_form(hom, N):
    """Layers normal to x_1 with random Lame moduli: the effective Mandel
    stiffness of the layered medium, every load case, both precisions."""
    d = len(N)
    m = d * (d + 1) // 2
    u = hi.uniform(61, 2 * N[0]).reshape(2, N[0])
    mu = 1.0 + 30.0 * u[0]
    lam = mu * (0.2 + 1.8 * u[1])
    A = np.stack([hi.laminate(N, lam), hi.laminate(N, mu)])
    ref = elastic_laminate_W(lam, mu, d)
    for prec, tol, bar in ((hom.FP64, 1e-12, 1e-10), (hom.MIXED, 1e-8, 1e-6)):
        W = hom.Cell(A, N, kind=hom.ELASTIC, prec=prec).solve(np.eye(m), tol=tol)["W"]
        assert rel(W, ref) < bar


@gpu
def test_elastic_homogeneous_and_bounds(hom):
    N = (31, 29, 27)
    A = np.stack([np.full(N, 1.7), np.full(N, 0.9)])
    W = hom.Cell(A, N, kind=hom.ELASTIC).solve(np.eye(6), tol=1e-10)["W"]
    assert np.abs(W - lame_stiffness(1.7, 0.9, 3)).max() < 1e-12
    A = lame_field(N, 97)
    W = hom.Cell(A, N, kind=hom.ELASTIC).solve(np.eye(6), tol=1e-10)["W"]
    Cs = np.stack([lame_stiffness(A[0][i], A[1][i], 3) for i in np.ndindex(*N)])
    assert np.linalg.eigvalsh(Cs.mean(axis=0) - W).min() > 0
    assert np.linalg.eigvalsh(W - np.linalg.inv(np.linalg.inv(Cs).mean(axis=0))).min() > 0


@gpu
def test_elastic_rejections(hom):
    A2 = np.stack([np.ones((9, 9)), np.ones((9, 9))])
    with pytest.raises(hom.HomError):
        hom.Cell(A2, (9, 9), kind=hom.ELASTIC, dual=True)
    with pytest.raises(hom.HomError):
        hom.Cell(np.stack([np.ones((9, 9)), -np.ones((9, 9))]), (9, 9), kind=hom.ELASTIC)
    with pytest.raises(hom.HomError):
        hom.Cell(np.stack([np.ones(9), np.ones(9)]), (9,), kind=hom.ELASTIC)
    srv = hom.Server(1 << 30)
    c = hom.Cell(A2, (9, 9), kind=hom.ELASTIC, prec=hom.MIXED)
    with pytest.raises(hom.HomError):
        srv.submit(c, np.eye(3))
    srv.close()
