"""The allocation-free operator apply (hom_apply_noalloc) against hom_apply:
same arguments, the library's fixed scratch as workspace.  Two calls in a row,
the second on a smaller input, so leftovers of the first call in the shared
scratch would show; FP64 to round-off, the FP32 arithmetic to the mixed bar."""
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


# (N, kind, scheme, load cases): a 3-D Ga cell with three load cases, then a
# smaller 2-D GaNi cell with one
CASES = [((17, 13, 15), 2, 1, 3), ((15, 13), 0, 0, 1)]


@gpu
@pytest.mark.parametrize("prec_name,bar", [("FP64", 1e-13), ("MIXED", 1e-6)])
def test_noalloc_apply_matches_apply(hom, prec_name, bar):
    import torch
    prec = getattr(hom, prec_name)
    for i, (N, kind, scheme, L) in enumerate(CASES):
        d = len(N)
        Q = tuple(2 * n - 1 for n in N) if scheme == hom.GA else N
        A = hi.random_spd_field(Q, kind, seed=40 + i, contrast=30.0)
        cell = hom.Cell(A, N, kind=kind, scheme=scheme)
        u = hi.normal(60 + i, L * d * int(np.prod(N))).reshape((L, d) + N)
        ut = torch.from_numpy(u).cuda()
        ref = cell.apply(ut, prec=prec).cpu().numpy()
        out = torch.full_like(ut, float("nan"))
        assert cell.apply_noalloc(ut, out, prec=prec) == 0
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        assert np.isfinite(got).all()
        assert rel(got, ref) <= bar, (prec_name, N, rel(got, ref))
        cell.close()


@gpu
def test_noalloc_rejects_a_workspace_above_the_scratch(hom):
    """1023^2 with three load cases needs ~151 MB of FP64 workspace: refused
    with HOM_ESCRATCH before anything runs; out is left untouched."""
    import torch
    N = (1023, 1023)
    cell = hom.Cell(np.ones(N), N)
    u = torch.zeros((3, 2) + N, dtype=torch.float64, device="cuda")
    out = torch.full_like(u, 7.0)
    assert cell.apply_noalloc(u, out) == -8
    torch.cuda.synchronize()
    assert bool((out == 7.0).all())
    # one load case fits
    assert cell.apply_noalloc(u[:1], out[:1]) == 0
    torch.cuda.synchronize()
    assert bool((out[:1] == 0.0).all())
    cell.close()
