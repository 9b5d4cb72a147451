"""Pins of the FP64 oracle to facts fixed by the paper and by mathematics,
independent of the oracle's own code paths.

Each test names the passage it follows.  None retypes the oracle's formula:
the checks are library routines (numpy FFT / dense linear algebra), closed
forms, invariants and brute-force solves.
"""
import numpy as np
import pytest

import hom_inputs as hi


def rand_field(shape, seed):
    return hi.normal(seed, int(np.prod(shape))).reshape(shape)


# ---------------------------------------------------------------- T1: DFT
@pytest.mark.parametrize("shape", [(7,), (5, 9), (3, 5, 7)])
def test_dft_matches_numpy_fft(oracle, shape):
    """DFT pair of Sec. 4.1: forward carries 1/n, inverse none; on FFT-order
    storage it equals the standard DFT (numpy) per axis."""
    z = rand_field(shape, 1) + 1j * rand_field(shape, 2)
    for ax in range(len(shape)):
        fwd = oracle.dft_axis(z, ax, -1)
        np.testing.assert_allclose(fwd, np.fft.fft(z, axis=ax) / shape[ax], atol=1e-14, rtol=0)
        inv = oracle.dft_axis(z, ax, +1)
        np.testing.assert_allclose(inv, np.fft.ifft(z, axis=ax) * shape[ax], atol=1e-13, rtol=0)


@pytest.mark.parametrize("shape", [(9, 5), (5, 3, 7)])
def test_dft_roundtrip_parseval_hermitian(oracle, shape):
    """Inverse after forward is the identity; Plancherel (Sec. 2) / isometry of
    Sec. 4.1: grid mean of u v equals sum of u^ conj(v^); real input gives a
    Hermitian spectrum."""
    u = rand_field(shape, 3)
    v = rand_field(shape, 4)
    U = oracle.dft_all(u, -1)
    V = oracle.dft_all(v, -1)
    np.testing.assert_allclose(oracle.dft_all(U, +1).real, u, atol=1e-13)
    np.testing.assert_allclose(np.mean(u * v), np.sum(U * np.conj(V)).real, atol=1e-14)
    # Hermitian: U(-k) = conj U(k); -k in FFT order is the index reversal mod n
    idx = np.ix_(*[(-np.arange(n)) % n for n in shape])
    np.testing.assert_allclose(U[idx], np.conj(U), atol=1e-15)


# ------------------------------------------------- T3: projection identities
@pytest.mark.parametrize("N,Y", [((9, 7), (0.5, 0.5)), ((5, 7, 3), (0.5, 0.5, 0.5)),
                                 ((7, 9), (0.5, 1.3))])
def test_projection_properties(oracle, N, Y):
    """Lemma on the discrete projection (Sec. 5.1) with A0 = I: G is
    idempotent, self-adjoint for the grid product, kills constants, leaves
    gradients of trigonometric polynomials unchanged, and its output is
    curl-free with zero mean."""
    d = len(N)
    c = oracle.Cell(np.ones(N), N, Y=Y)
    u = rand_field((d,) + N, 11)
    v = rand_field((d,) + N, 12)
    Gu = c.apply_G(u)
    Gv = c.apply_G(v)
    np.testing.assert_allclose(c.apply_G(Gu), Gu, atol=1e-13)
    np.testing.assert_allclose(np.mean(Gu * v), np.mean(u * Gv), atol=1e-14)
    const = np.stack([np.full(N, 1.0 + a) for a in range(d)])
    np.testing.assert_allclose(c.apply_G(const), 0.0, atol=1e-14)
    np.testing.assert_allclose(Gu.reshape(d, -1).mean(axis=1), 0.0, atol=1e-14)
    # gradient of a random real trigonometric polynomial phi (numpy FFT synthesis)
    phi_hat = np.fft.fftn(rand_field(N, 13))
    ks = np.meshgrid(*[hi.signed_index(n) for n in N], indexing="ij")
    grad = np.stack([np.fft.ifftn(1j * np.pi * (ks[a] / Y[a]) * phi_hat).real for a in range(d)])
    np.testing.assert_allclose(c.apply_G(grad), grad, atol=1e-12 * np.abs(grad).max())
    # curl-free: xi_a e^_b = xi_b e^_a for the spectrum of G u
    Ghat = np.stack([np.fft.fftn(Gu[a]) for a in range(d)])
    for a in range(d):
        for b in range(a + 1, d):
            lhs = (ks[a] / Y[a]) * Ghat[b]
            rhs = (ks[b] / Y[b]) * Ghat[a]
            np.testing.assert_allclose(lhs, rhs, atol=1e-11)


# ----------------------------------------------------- T2: homogeneous cell
@pytest.mark.parametrize("kind", [0, 1, 2])
@pytest.mark.parametrize("N", [(5, 7), (3, 5, 5)])
def test_homogeneous_cell_recovers_A(oracle, kind, N):
    """Lemma 1 (iv): G kills constant fields, so for constant SPD A the
    right-hand side -G A E vanishes (up to the DFT's rounding), the
    fluctuation is zero and the homogenized coefficient is A itself."""
    d = len(N)
    A1 = hi.random_spd_field((1,) * d, kind, seed=21, contrast=5.0)
    A = np.broadcast_to(A1.reshape(A1.shape[:A1.ndim - d] + (1,) * d),
                        A1.shape[:A1.ndim - d] + N).copy()
    c = oracle.Cell(A, N, kind=kind)
    x, W, J, its = c.solve(np.eye(d), tol=1e-10)
    assert np.abs(x).max() < 1e-14
    if kind == 0:
        Afull = A1.reshape(-1)[0] * np.eye(d)
    elif kind == 1:
        Afull = np.diag(A1.reshape(d))
    else:
        v = A1.reshape(-1)
        idx = {1: [(0, 0)], 2: [(0, 0), (1, 1), (0, 1)],
               3: [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]}[d]
        Afull = np.zeros((d, d))
        for t, (a, b) in enumerate(idx):
            Afull[a, b] = Afull[b, a] = v[t]
    np.testing.assert_allclose(W, Afull, rtol=1e-14, atol=1e-14)


# ---------------------------------------------------------- T4: laminates
@pytest.mark.parametrize("N", [(9, 7), (7, 5, 5), (15,)])
def test_laminate_closed_form(oracle, N):
    """A = a(x_1) I: the across-layer entry is the harmonic mean of the grid
    samples, along-layer entries the arithmetic mean, off-diagonals zero
    (the exact discrete solution has A e constant across the layers)."""
    d = len(N)
    a = 1.0 + 99.0 * hi.uniform(31, N[0])
    A = hi.laminate(N, a)
    c = oracle.Cell(A, N)
    x, W, J, its = c.solve(np.eye(d), tol=1e-13)
    ref = np.diag([1.0 / np.mean(1.0 / a)] + [np.mean(a)] * (d - 1))
    np.testing.assert_allclose(W, ref, rtol=1e-12, atol=1e-12 * np.mean(a))


@pytest.mark.parametrize("n", [3, 5, 9, 15, 31])
def test_cosine_laminate_trapezoid(oracle, n):
    """a = 2 + cos(2 pi x_1): the harmonic mean of N grid samples equals
    sqrt(3) (1 - r^N) / (1 + r^N), r = sqrt(3) - 2 (trapezoid rule on the
    Poisson kernel expansion of 1 / (2 + cos))."""
    N = (n, 5)
    x1 = hi.coords(N)[0]
    a = 2.0 + np.cos(2 * np.pi * x1)
    c = oracle.Cell(hi.laminate(N, a), N)
    _, W, _, _ = c.solve(np.eye(2), tol=1e-14)
    r = np.sqrt(3.0) - 2.0
    np.testing.assert_allclose(W[0, 0], np.sqrt(3.0) * (1 - r ** n) / (1 + r ** n), rtol=1e-14)
    np.testing.assert_allclose(W[1, 1], 2.0, rtol=1e-15)


# ------------------------------------------------- T5: dense brute force
def _dense_G(c, d, N):
    n = d * int(np.prod(N))
    G = np.empty((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        G[:, j] = c.apply_G(e.reshape((d,) + N)).reshape(-1)
    return G


def _dense_op(c, d, N):
    n = d * int(np.prod(N))
    K = np.empty((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        K[:, j] = c.apply_GA(e.reshape((d,) + N)).reshape(-1)
    return K


def _A_matrix_at(A, kind, d, p):
    """d x d coefficient at flat grid point p from a (nA, npts) array."""
    if kind == 0:
        return A[0, p] * np.eye(d)
    if kind == 1:
        return np.diag(A[:, p])
    idx = {1: [(0, 0)], 2: [(0, 0), (1, 1), (0, 1)],
           3: [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]}[d]
    M = np.zeros((d, d))
    for t, (a, b) in enumerate(idx):
        M[a, b] = M[b, a] = A[t, p]
    return M


def fourier_galerkin_dense(A, kind, N, scheme, E, Y=None):
    """Dense Fourier-Galerkin solve of the discrete cell problem, independent
    of the oracle: unknowns c(k), k in Z_N \\ {0}, with e^(k) = n(k) c(k),
    n = xi / |xi|; K_km = n(k)^T A^(k - m) n(m), b_k = -n(k)^T A^(k) E, where
    A^ is the DFT (numpy) of A on the quadrature grid Q and k - m is taken
    mod Q.  Returns the fluctuation on the N grid and W over the Q grid."""
    N = tuple(N)
    d = len(N)
    Y = (0.5,) * d if Y is None else Y
    Q = tuple(2 * n - 1 for n in N) if scheme == 1 else N
    nA = A.shape[0] if A.ndim == d + 1 else 1
    A = A.reshape((nA,) + Q)
    Ahat = np.stack([np.fft.fftn(A[t]) / np.prod(Q) for t in range(nA)])
    ks = np.array(list(np.ndindex(*N)))
    kk = np.stack([hi.signed_index(n)[ks[:, a]] for a, n in enumerate(N)], axis=1)
    nz = np.any(kk != 0, axis=1)
    kk = kk[nz]
    xi = kk / np.array(Y)
    nv = xi / np.linalg.norm(xi, axis=1, keepdims=True)
    m = len(kk)

    def Ahat_mat(j):  # j: (..., d) signed integer differences
        idx = tuple(np.mod(j[..., a], Q[a]) for a in range(d))
        vals = Ahat[(slice(None),) + idx]           # (nA, ...)
        M = np.zeros(j.shape[:-1] + (d, d), dtype=complex)
        if kind == 0:
            for a in range(d):
                M[..., a, a] = vals[0]
        elif kind == 1:
            for a in range(d):
                M[..., a, a] = vals[a]
        else:
            ids = {1: [(0, 0)], 2: [(0, 0), (1, 1), (0, 1)],
                   3: [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]}[d]
            for t, (a, b) in enumerate(ids):
                M[..., a, b] = vals[t]
                M[..., b, a] = vals[t]
        return M

    diff = kk[:, None, :] - kk[None, :, :]
    Am = Ahat_mat(diff)                                   # (m, m, d, d)
    K = np.einsum("ka,kmab,mb->km", nv, Am, nv)
    x_out, W = [], None
    E = np.atleast_2d(E)
    fields = []
    for El in E:
        b = -np.einsum("ka,kab,b->k", nv, Ahat_mat(kk), El)
        cc = np.linalg.solve(K, b)
        spec = np.zeros((d,) + N, dtype=complex)
        for t in range(m):
            pos = tuple(int(kk[t, a]) % N[a] for a in range(d))
            spec[(slice(None),) + pos] = nv[t] * cc[t]
        x = np.stack([np.fft.ifftn(spec[a]).real * np.prod(N) for a in range(d)])
        x_out.append(x)
        # total strain on Q: pad the spectrum to Q and synthesise
        specQ = np.zeros((d,) + Q, dtype=complex)
        for t in range(m):
            pos = tuple(int(kk[t, a]) % Q[a] for a in range(d))
            specQ[(slice(None),) + pos] = nv[t] * cc[t]
        eQ = np.stack([np.fft.ifftn(specQ[a]).real * np.prod(Q) + El[a] for a in range(d)])
        fields.append(eQ.reshape(d, -1))
    Aflat = A.reshape(nA, -1)
    L = len(E)
    W = np.zeros((L, L))
    nq = Aflat.shape[1]
    for p in range(nq):
        Ap = _A_matrix_at(Aflat, kind, d, p)
        for l in range(L):
            for mm in range(L):
                W[l, mm] += fields[l][:, p] @ Ap @ fields[mm][:, p]
    return np.stack(x_out), W / nq


CASES = [((3, 3), 0), ((5, 5), 1), ((7, 5), 2), ((3, 5), 0), ((3, 3, 3), 1), ((5, 3, 3), 2)]


@pytest.mark.parametrize("N,kind", CASES)
@pytest.mark.parametrize("scheme", [0, 1])
def test_dense_fourier_galerkin(oracle, N, kind, scheme):
    """Brute force (ii): the Galerkin system assembled densely in the basis
    n(k) phi_k of E_N (Sec. 4.2-4.3; for GaNi A^(k-m) wraps mod N, the
    aliasing of Q_N; for Ga on the 2N-1 grid it never wraps) and solved by LU
    gives the same fluctuation and W as the oracle's CG."""
    d = len(N)
    Q = tuple(2 * n - 1 for n in N) if scheme == 1 else N
    A = hi.random_spd_field(Q, kind, seed=41 + kind, contrast=20.0)
    c = oracle.Cell(A, N, kind=kind, scheme=scheme)
    x, W, J, its = c.solve(np.eye(d), tol=1e-14)
    xr, Wr = fourier_galerkin_dense(A, kind, N, scheme, np.eye(d))
    np.testing.assert_allclose(x, xr, atol=1e-11 * max(1.0, np.abs(xr).max()))
    np.testing.assert_allclose(W, Wr, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("N,kind", CASES[:4])
@pytest.mark.parametrize("scheme", [0, 1])
def test_dense_realspace(oracle, N, kind, scheme):
    """Brute force (i): with the oracle's operator K = G A assembled column by
    column and G the orthogonal projection, (K G + I - G) x = -K E is SPD on
    the grid and its LU solution is the CG solution (Sec. 5.3, the CG Lemma)."""
    d = len(N)
    Q = tuple(2 * n - 1 for n in N) if scheme == 1 else N
    A = hi.random_spd_field(Q, kind, seed=51 + kind, contrast=30.0)
    c = oracle.Cell(A, N, kind=kind, scheme=scheme)
    G = _dense_G(c, d, N)
    K = _dense_op(c, d, N)
    n = G.shape[0]
    for E in np.eye(d):
        Ef = np.repeat(E, int(np.prod(N)))
        M = K @ G + np.eye(n) - G
        x_ref = np.linalg.solve(M, -K @ Ef)
        x, it, rr = c.cg(E, tol=1e-14)
        np.testing.assert_allclose(x.reshape(-1), x_ref, atol=1e-12 * max(1, np.abs(x_ref).max()))
        assert it <= n
        # the projected operator is symmetric on E_N: (K G) restricted = G K G
        np.testing.assert_allclose(G @ K @ G, (G @ K @ G).T, atol=1e-12 * np.abs(K).max())


# --------------------------------------------- warm start (Sec. 5.3, CG Lemma)
@pytest.mark.parametrize("scheme", [0, 1])
def test_warm_start(oracle, scheme):
    """CG keeps its iterates in E_N and the discrete solution is unique
    (Sec. 5.2-5.3), so a warm start enters through its E_N part.  The stopping
    test is relative to ||b|| (the cold start's initial residual).  (i) From
    the solution of the dense Fourier-Galerkin system (no CG) the test holds at
    once: 0 iterations, the same field.  (ii) From a gradient field plus
    constants and a divergence-free field (both outside E_N) CG ends at that
    same solution: the part outside E_N is projected away."""
    N = (7, 5)
    d, kind = 2, 2
    Q = tuple(2 * n - 1 for n in N) if scheme == 1 else N
    A = hi.random_spd_field(Q, kind, seed=73, contrast=20.0)
    c = oracle.Cell(A, N, kind=kind, scheme=scheme)
    E = np.array([1.0, -0.4])
    xr = fourier_galerkin_dense(A, kind, N, scheme, E[None])[0][0]
    scale = np.abs(xr).max()
    x, it, rr = c.cg(E, tol=1e-10, x0=xr)
    assert it == 0
    np.testing.assert_allclose(x, xr, atol=1e-13 * scale)
    ks = np.meshgrid(*[hi.signed_index(n) for n in N], indexing="ij")
    xi = [2.0 * k for k in ks]   # xi = k / Y with Y = 1/2
    phi = np.fft.fftn(rand_field(N, 74))
    psi = np.fft.fftn(rand_field(N, 75))
    grad = np.stack([np.fft.ifftn(1j * xi[a] * phi).real for a in range(d)])
    rot = np.stack([np.fft.ifftn(-1j * xi[1] * psi).real, np.fft.ifftn(1j * xi[0] * psi).real])
    x0 = grad + rot + np.array([0.7, -1.3])[:, None, None]
    np.testing.assert_allclose(c.apply_G(rot), 0.0, atol=1e-12 * np.abs(rot).max())
    x, it, rr = c.cg(E, tol=1e-13, x0=x0)
    assert it > 0
    np.testing.assert_allclose(x, xr, atol=1e-10 * scale)


# ------------------------------------------------------- T6: A_H structure
@pytest.mark.parametrize("N,kind,scheme", [((9, 7), 0, 0), ((7, 7), 2, 0), ((5, 5, 5), 1, 0),
                                           ((5, 7), 2, 1), ((3, 5, 3), 0, 1)])
def test_AH_symmetric_spd_voigt_reuss(oracle, N, kind, scheme):
    """W = A_H is symmetric, positive definite and lies between the Reuss and
    Voigt means of the quadrature-grid samples in the Loewner order (energy
    principles of the conforming discrete problem, Sec. 3-5)."""
    d = len(N)
    Q = tuple(2 * n - 1 for n in N) if scheme == 1 else N
    A = hi.random_spd_field(Q, kind, seed=61 + kind, contrast=50.0)
    c = oracle.Cell(A, N, kind=kind, scheme=scheme)
    _, W, J, _ = c.solve(np.eye(d), tol=1e-13)
    np.testing.assert_allclose(W, W.T, rtol=1e-12, atol=1e-12)
    Aflat = A.reshape(A.shape[0] if A.ndim == d + 1 else 1, -1)
    mats = np.stack([_A_matrix_at(Aflat, kind, d, p) for p in range(Aflat.shape[1])])
    voigt = mats.mean(axis=0)
    reuss = np.linalg.inv(np.linalg.inv(mats).mean(axis=0))
    assert np.linalg.eigvalsh(W).min() > 0
    assert np.linalg.eigvalsh(voigt - W).min() >= -1e-12 * np.abs(W).max()
    assert np.linalg.eigvalsh(W - reuss).min() >= -1e-12 * np.abs(W).max()
    # energy and mean flux agree at convergence (Galerkin orthogonality)
    np.testing.assert_allclose(W, J, rtol=1e-10, atol=1e-10)


def test_square_inclusion_symmetry(oracle):
    """Centred square on the origin-symmetric grid (A4): A_H is isotropic
    with a vanishing off-diagonal entry."""
    w = hi.cfg1_square()
    c = oracle.Cell(w.A, w.N)
    _, W, _, _ = c.solve(np.eye(2), tol=1e-13)
    np.testing.assert_allclose(W[0, 0], W[1, 1], rtol=1e-13)
    assert abs(W[0, 1]) < 1e-13
    assert 1.0 < W[0, 0] < 10.0


# ------------------------------------------------- T8: L-SD invariance
@pytest.mark.parametrize("lam", [0.5, 1.0, 7.3])
def test_lsd_cg_independent_of_reference(oracle, lam):
    """Sec. 5.3: CG on the discrete Lippmann-Schwinger system with A0 = lambda I
    gives e = E + the solution of G A e~ = -G A E for every lambda."""
    N = (9, 7)
    A = hi.random_spd_field(N, 0, seed=71, contrast=10.0)
    c = oracle.Cell(A, N)
    E = np.array([0.3, -1.1])
    x, _, _ = c.cg(E, tol=1e-14)
    e, _ = c.cg_lsd(E, lam, tol=1e-14)
    np.testing.assert_allclose(e, x + E[:, None, None], atol=1e-12)


# --------------------------------------------------- T10 / T11
def test_apriori_bound_and_ms_limit(oracle):
    """Moulinec-Suquet fixed point (Sec. 5.3) with lambda = (c_A + C_A)/2
    converges to the same e; the fluctuation obeys ||e~|| <= rho_A ||E||
    (the a-priori bound of the regularity appendix)."""
    N = (7, 9)
    A = hi.random_spd_field(N, 0, seed=81, contrast=10.0)
    c = oracle.Cell(A, N)
    E = np.array([1.0, 0.5])
    x, _, _ = c.cg(E, tol=1e-14)
    lam = 0.5 * (A.min() + A.max())
    e, it = c.ms(E, lam, tol=1e-13)
    np.testing.assert_allclose(e, x + E[:, None, None], atol=1e-11)
    rho = A.max() / A.min()
    assert np.sqrt(np.mean(x ** 2) * 2) <= rho * np.linalg.norm(E)
    # CG needs far fewer iterations than the Neumann series (Sec. 5.3)
    _, it_cg, _ = c.cg(E, tol=1e-13)
    assert it_cg < it


# ---------------------------------------------------------- T9: Ga checks
def test_ga_cosine_laminate_monotone(oracle):
    """Ga with A = 2 + cos(2 pi x_1) sampled on the 2N-1 grid is the exact
    conforming Galerkin method for that coefficient (the interpolant of a
    degree-1 trigonometric polynomial is itself): the along-layer entry is 2
    exactly and the across-layer entry decreases monotonically to sqrt(3)
    from above as the nested trial spaces grow (Cea, Sec. 4.2)."""
    prev = np.inf
    vals = []
    for n in (3, 5, 9, 15):
        N = (n, 3)
        M = (2 * n - 1, 5)
        x1 = hi.coords(M)[0]
        A = hi.laminate(M, 2.0 + np.cos(2 * np.pi * x1))
        c = oracle.Cell(A, N, scheme=1)
        _, W, _, _ = c.solve(np.eye(2), tol=1e-14)
        np.testing.assert_allclose(W[1, 1], 2.0, rtol=1e-14)
        assert W[0, 0] >= np.sqrt(3.0) - 1e-14
        assert W[0, 0] < prev
        prev = W[0, 0]
        vals.append(W[0, 0] - np.sqrt(3.0))
    assert vals[-1] < 1e-7
    assert vals[0] > 1e-3


def test_ga_laminate_bounds(oracle):
    """Ga laminate sampled on the 2N-1 grid: along-layer entry = arithmetic
    mean of the M samples; across-layer entry >= harmonic mean of them."""
    N = (7, 5)
    M = (13, 9)
    a = 1.0 + 30.0 * hi.uniform(91, M[0])
    c = oracle.Cell(hi.laminate(M, a), N, scheme=1)
    _, W, _, _ = c.solve(np.eye(2), tol=1e-14)
    np.testing.assert_allclose(W[1, 1], a.mean(), rtol=1e-13)
    assert W[0, 0] >= 1.0 / np.mean(1.0 / a) - 1e-12
    assert abs(W[0, 1]) < 1e-12


def test_cg_iterations_grow_sublinearly_with_contrast(oracle):
    """Sec. 5.3: CG iteration counts grow like sqrt(rho_A) (loose check: going
    from contrast 10 to 1000 multiplies them by far less than 100)."""
    N = (31, 31)
    its = []
    for rho in (10.0, 1000.0):
        A = hi.bernoulli_majority(N, 0.4, 3, rho, 1.0, seed=7)
        c = oracle.Cell(A, N)
        _, it, _ = c.cg([1.0, 0.0], tol=1e-8)
        its.append(it)
    assert its[1] < 20 * its[0]


def test_invalid_inputs_rejected(oracle):
    from oracle.oracle import OracleError
    with pytest.raises(OracleError):      # even N violates (A4)
        oracle.Cell(np.ones((4, 5)), (4, 5)).apply_G(np.zeros((2, 4, 5)))
    c = oracle.Cell(np.ones((5, 5)), (5, 5))
    with pytest.raises(OracleError):
        c.cg([1.0, 0.0], tol=-1.0)


def _loglog_slope(x, y):
    return float(np.polyfit(np.log(x), np.log(y), 1)[0])


def test_ms_iterations_linear_cg_sqrt_in_contrast(oracle):
    """Sec. 5.3: the Moulinec-Suquet scheme with lambda = (c_A + C_A)/2
    contracts by (rho_A - 1)/(rho_A + 1) per step, so its step count to a
    fixed tolerance grows like rho_A; CG's like sqrt(rho_A).  Fitted
    log-log slopes over rho_A = 10, 100, 1000 on a two-phase pixel cell; MS
    never beats the contraction bound."""
    N = (15, 15)
    tol = 1e-4
    rhos = [10.0, 100.0, 1000.0]
    ms, cg = [], []
    for rho in rhos:
        A = hi.bernoulli_majority(N, 0.4, 3, rho, 1.0, seed=7)
        c = oracle.Cell(A, N)
        E = np.array([1.0, 0.0])
        _, it_cg, _ = c.cg(E, tol=tol)
        _, it_ms = c.ms(E, 0.5 * (1.0 + rho), tol=tol, max_iter=200000)
        cg.append(it_cg)
        ms.append(it_ms)
        # ||r_i|| <= q^i ||b|| in the energy-free bound: i >= log(tol) / log(q)
        # steps are not needed beyond the bound (plus the conditioning factor)
        q = (rho - 1.0) / (rho + 1.0)
        assert it_ms <= np.log(tol / np.sqrt(rho)) / np.log(q) + 2
    assert _loglog_slope(rhos, ms) > 0.75
    assert _loglog_slope(rhos, cg) < 0.5


# ------------------------------- Ga with exact integration (Sec. 4.2-4.3)
def test_ga_exact_laminate_step(oracle):
    """A layer |x_1| < 0.15 of contrast 100 given by its Fourier coefficients:
    Ga on the M-grid samples of the truncated series integrates A u.v exactly
    (u.v lies in T_M), so the along-layer entry is the exact volume average
    (vf 0.3, no voxel count) for every N, and the across-layer entry bounds
    the exact harmonic mean from above and decreases as the nested trial
    spaces grow (Cea).  The samples dip below 0 near the jumps; the form on
    T_N is still that of the positive coefficient."""
    harm = 1.0 / (0.3 / 100.0 + 0.7 / 1.0)
    prev = np.inf
    for n in (3, 5, 9, 17, 33):
        N = (n, 3)
        A = hi.laminate_step_trig(N, 0.3, 100.0, 1.0)
        c = oracle.Cell(A, N, scheme=1)
        _, W, _, _ = c.solve(np.eye(2), tol=1e-14)
        np.testing.assert_allclose(W[1, 1], 1.0 + 99.0 * 0.3, rtol=1e-13)
        assert abs(W[0, 1]) < 1e-11
        assert W[0, 0] >= harm * (1 - 1e-12)
        assert W[0, 0] < prev
        prev = W[0, 0]
    assert A.min() < 0.0
    assert prev < 1.1 * harm


def test_ga_exact_square_bounds(oracle):
    """Centred square of vf 1/4 and contrast 100 by its Fourier coefficients:
    W is symmetric under the square's symmetries (W_11 = W_22, W_12 = 0),
    lies between the Reuss and Voigt means of the exact phases and
    decreases with N (conforming and nested)."""
    f, a1, a0 = 0.25, 100.0, 1.0
    voigt, reuss = f * a1 + (1 - f) * a0, 1.0 / (f / a1 + (1 - f) / a0)
    prev = np.inf
    for n in (5, 9, 17):
        A = hi.square_inclusion_trig((n, n), 0.25, a1, a0)
        c = oracle.Cell(A, (n, n), scheme=1)
        _, W, _, _ = c.solve(np.eye(2), tol=1e-14)
        np.testing.assert_allclose(W[0, 0], W[1, 1], rtol=1e-12)
        assert abs(W[0, 1]) < 1e-11 * W[0, 0]
        assert reuss < W[0, 0] < voigt
        assert W[0, 0] < prev
        prev = W[0, 0]


def test_ga_exact_sphere_above_hashin_shtrikman(oracle):
    """A centred ball (r = 0.25, contrast 10) by its Fourier coefficients:
    W is isotropic (cubic symmetry of the cell), decreases with N, and stays
    above the Hashin-Shtrikman lower bound of the exact volume fraction,
    which bounds the exact homogenized coefficient that Ga bounds from above."""
    r, a1, a0 = 0.25, 10.0, 1.0
    f = 4.0 / 3.0 * np.pi * r ** 3
    hs = a0 + f / (1.0 / (a1 - a0) + (1.0 - f) / (3.0 * a0))
    prev = np.inf
    for n in (3, 5, 7):
        N = (n, n, n)
        A = hi.inclusions_trig(N, 1, r, a1, a0, centres=[[0.5, 0.5, 0.5]])
        c = oracle.Cell(A, N, scheme=1)
        _, W, _, _ = c.solve(np.eye(3), tol=1e-14)
        np.testing.assert_allclose(np.diag(W), W[0, 0], rtol=1e-11)
        assert np.abs(W - np.diag(np.diag(W))).max() < 1e-11 * W[0, 0]
        assert W[0, 0] > hs
        assert W[0, 0] < prev
        prev = W[0, 0]


# ------------------------- dual (flux) formulation on J_N (Sec. 5.1, Sec. 6)
@pytest.mark.parametrize("N", [(9, 7), (5, 7, 3)])
def test_dual_projection_helmholtz(oracle, N):
    """The discrete Helmholtz decomposition (Sec. 5.1): G u + G_dual u +
    mean(u) = u; G_dual is idempotent, orthogonal to G, and its output is
    divergence-free (xi . j^ = 0) with zero mean."""
    d = len(N)
    cp = oracle.Cell(np.ones(N), N)
    cd = oracle.Cell(np.ones(N), N, dual=True)
    u = rand_field((d,) + N, 21)
    v = rand_field((d,) + N, 22)
    Gu, Du = cp.apply_G(u), cd.apply_G(u)
    mean = u.reshape(d, -1).mean(axis=1).reshape((d,) + (1,) * d)
    np.testing.assert_allclose(Gu + Du + mean, u, atol=1e-13)
    np.testing.assert_allclose(cd.apply_G(Du), Du, atol=1e-13)
    assert abs(np.mean(Du * cp.apply_G(v))) < 1e-14
    ks = np.meshgrid(*[hi.signed_index(n) for n in N], indexing="ij")
    div = sum(2.0 * ks[a] * np.fft.fftn(Du[a]) for a in range(d))
    assert np.abs(div).max() < 1e-11 * np.abs(np.fft.fftn(Du[0])).max()


@pytest.mark.parametrize("N", [(15, 7), (9, 5, 7)])
def test_dual_laminate_closed_form(oracle, N):
    """Dual problem with the resistivity B = 1/a(x_1) of a laminate: the flux
    along x_1 must be constant and across it is free, so the dual energy is
    diag(<1/a>, 1/<a>, ...) and its inverse the primal closed form."""
    d = len(N)
    a = 1.0 + 50.0 * hi.uniform(31, N[0])
    c = oracle.Cell(hi.laminate(N, 1.0 / a), N, dual=True)
    _, W, _, _ = c.solve(np.eye(d), tol=1e-14)
    ref = np.diag([np.mean(1.0 / a)] + [1.0 / np.mean(a)] * (d - 1))
    np.testing.assert_allclose(W, ref, rtol=1e-12, atol=1e-13)


def test_dual_two_sided_bounds_exact_square(oracle):
    """Ga with both coefficients integrated exactly (Fourier-given square of
    contrast 20: A for the primal, B = A^-1 for the dual): the primal energy
    bounds A_H from above and the inverse of the dual energy from below
    (Sec. 6), and the gap shrinks as the nested trial spaces grow."""
    a1, a0 = 20.0, 1.0
    gaps = []
    for n in (5, 9, 17):
        N = (n, n)
        A = hi.square_inclusion_trig(N, 0.25, a1, a0)
        B = hi.square_inclusion_trig(N, 0.25, 1.0 / a1, 1.0 / a0)
        _, Wp, _, _ = oracle.Cell(A, N, scheme=1).solve(np.eye(2), tol=1e-14)
        _, Wd, _, _ = oracle.Cell(B, N, scheme=1, dual=True).solve(np.eye(2), tol=1e-14)
        lower = np.linalg.inv(Wd)
        assert np.linalg.eigvalsh(Wp - lower).min() > 0
        gaps.append(Wp[0, 0] - lower[0, 0])
    assert gaps[2] < gaps[1] < gaps[0]


# ------------------- linear elasticity (the extension named in Sec. 6)
from elastic_ref import (elastic_laminate_W, from_mandel, lame_field, lame_stiffness,  # noqa: E402
                         mandel_pairs, to_mandel)


def sym_grad_mandel(U, Y=None):
    """Mandel strain of the trigonometric displacement U [d][N] by numpy FFT
    differentiation (d/dx_a <-> 2 pi i k_a / (2 Y_a))."""
    d = U.shape[0]
    N = U.shape[1:]
    Y = (0.5,) * d if Y is None else Y
    ks = np.meshgrid(*[hi.signed_index(n) for n in N], indexing="ij")
    Uh = np.stack([np.fft.fftn(U[a]) for a in range(d)])
    G = np.zeros((d, d) + tuple(N))
    for a in range(d):
        for b in range(d):
            G[a, b] = np.fft.ifftn(1j * np.pi * ks[b] / Y[b] * Uh[a]).real
    return to_mandel(0.5 * (G + G.transpose((1, 0) + tuple(range(2, 2 + d)))), d)


@pytest.mark.parametrize("N,Y", [((9, 7), None), ((5, 7, 3), None), ((7, 5), (0.5, 0.8)),
                                 ((5, 3, 5), (0.7, 0.5, 0.4))])
def test_elastic_projection_properties(oracle, N, Y):
    """G onto compatible strains: idempotent, self-adjoint in the grid inner
    product, zero on constants, the identity on symmetric gradients of
    trigonometric displacements (numpy FFT), and its output satisfies the
    compatibility condition inc(Z) = xi x Z x xi = 0 at every frequency."""
    d = len(N)
    m = d * (d + 1) // 2
    c = oracle.Cell(lame_field(N, 3), N, kind=oracle.ELASTIC, Y=Y)
    u = rand_field((m,) + N, 51)
    v = rand_field((m,) + N, 52)
    Gu, Gv = c.apply_G(u), c.apply_G(v)
    np.testing.assert_allclose(c.apply_G(Gu), Gu, atol=1e-13)
    assert abs(np.mean(Gu * v) - np.mean(u * Gv)) < 1e-14
    const = np.ones((m,) + N) * np.arange(1, m + 1).reshape((m,) + (1,) * d)
    assert np.abs(c.apply_G(const)).max() < 1e-13
    U = rand_field((d,) + N, 53)
    for a in range(d):
        U[a] = np.fft.ifftn(np.fft.fftn(U[a])).real
    eps = sym_grad_mandel(U, Y)
    np.testing.assert_allclose(c.apply_G(eps), eps, atol=1e-12 * np.abs(eps).max())
    Zh = from_mandel(np.stack([np.fft.fftn(Gu[t]) for t in range(m)]), d)
    Yv = (0.5,) * d if Y is None else Y
    ks = [k / Yv[a] for a, k in enumerate(np.meshgrid(*[hi.signed_index(n) for n in N],
                                                      indexing="ij"))]
    if d == 2:
        inc = ks[1] ** 2 * Zh[0, 0] + ks[0] ** 2 * Zh[1, 1] - 2 * ks[0] * ks[1] * Zh[0, 1]
    else:
        eps3 = np.zeros((3, 3, 3))
        eps3[0, 1, 2] = eps3[1, 2, 0] = eps3[2, 0, 1] = 1.0
        eps3[0, 2, 1] = eps3[2, 1, 0] = eps3[1, 0, 2] = -1.0
        K = np.stack(ks).astype(float)
        inc = np.einsum("ikl,jmn,k...,m...,ln...->ij...", eps3, eps3, K, K, Zh)
    assert np.abs(inc).max() < 1e-11 * np.abs(Zh).max()


@pytest.mark.parametrize("N", [(7, 5), (5, 3, 5)])
def test_elastic_homogeneous_cell(oracle, N):
    """Constant Lame moduli: the fluctuation vanishes and the energy matrix of
    the unit Mandel strains is the stiffness itself."""
    d = len(N)
    m = d * (d + 1) // 2
    A = np.stack([np.full(N, 1.7), np.full(N, 0.9)])
    x, W, J, its = oracle.Cell(A, N, kind=oracle.ELASTIC).solve(np.eye(m), tol=1e-12)
    np.testing.assert_allclose(W, lame_stiffness(1.7, 0.9, d), atol=1e-13)
    assert np.abs(x).max() < 1e-13


@pytest.mark.parametrize("N", [(15, 7), (9, 5, 7)])
def test_elastic_laminate_closed_form(oracle, N):
    d = len(N)
    m = d * (d + 1) // 2
    u = hi.uniform(61, 2 * N[0]).reshape(2, N[0])
    mu = 1.0 + 30.0 * u[0]
    lam = mu * (0.2 + 1.8 * u[1])
    A = np.stack([hi.laminate(N, lam), hi.laminate(N, mu)])
    _, W, _, _ = oracle.Cell(A, N, kind=oracle.ELASTIC).solve(np.eye(m), tol=1e-14)
    np.testing.assert_allclose(W, elastic_laminate_W(lam, mu, d), rtol=1e-11, atol=1e-11)


def elastic_fourier_galerkin_dense(A, N, scheme, E):
    """Dense Galerkin solve in displacement form, independent of the oracle:
    unknowns u^(k) in C^d for k in Z_N \\ {0}, strain^(k) = B(k) u^(k) with
    B(k) u = Mandel(sym(xi (x) u)) (not normalised), K_km = B(k)^T C^(k - m)
    B(m) and b_k = -B(k)^T C^(k) E with C^ the numpy DFT of the Mandel
    stiffness field on Q (k - m mod Q).  Returns W over the Q grid."""
    N = tuple(N)
    d = len(N)
    m = d * (d + 1) // 2
    Q = tuple(2 * n - 1 for n in N) if scheme == 1 else N
    Cx = np.zeros((m, m) + Q)
    for idx in np.ndindex(*Q):
        Cx[(slice(None), slice(None)) + idx] = lame_stiffness(A[0][idx], A[1][idx], d)
    Ch = np.fft.fftn(Cx, axes=tuple(range(2, 2 + d))) / np.prod(Q)
    ks = np.array(list(np.ndindex(*N)))
    kk = np.stack([hi.signed_index(n)[ks[:, a]] for a, n in enumerate(N)], axis=1)
    kk = kk[np.any(kk != 0, axis=1)]
    xi = kk / 0.5
    B = np.zeros((len(kk), m, d))
    for p in range(d):
        for t, (a, b) in enumerate(mandel_pairs(d)):
            f = 1.0 if a == b else np.sqrt(2.0)
            B[:, t, p] = f * 0.5 * (xi[:, a] * (b == p) + xi[:, b] * (a == p))

    def Cmat(j):
        idx = tuple(np.mod(j[..., a], Q[a]) for a in range(d))
        return np.moveaxis(Ch[(slice(None), slice(None)) + idx], (0, 1), (-2, -1))

    K = np.einsum("kta,kmts,msb->kamb", B, Cmat(kk[:, None, :] - kk[None, :, :]), B)
    n = len(kk) * d
    K = K.reshape(n, n)
    fields = []
    for El in np.atleast_2d(E):
        rhs = -np.einsum("kta,kts,s->ka", B, Cmat(kk), El).reshape(n)
        uh = np.linalg.solve(K, rhs).reshape(len(kk), d)
        specQ = np.zeros((m,) + Q, dtype=complex)
        for t in range(len(kk)):
            pos = tuple(int(kk[t, a]) % Q[a] for a in range(d))
            specQ[(slice(None),) + pos] = B[t] @ uh[t]
        eQ = np.stack([np.fft.ifftn(specQ[s]).real * np.prod(Q) + El[s] for s in range(m)])
        fields.append(eQ.reshape(m, -1))
    Cf = Cx.reshape(m, m, -1)
    L = len(fields)
    W = np.zeros((L, L))
    for l in range(L):
        for k2 in range(L):
            W[l, k2] = np.mean(np.einsum("sp,stp,tp->p", fields[l], Cf, fields[k2]))
    return W


@pytest.mark.parametrize("N", [(3, 5), (5, 5), (3, 3, 3)])
@pytest.mark.parametrize("scheme", [0, 1])
def test_elastic_dense_fourier_galerkin(oracle, N, scheme):
    """The oracle's real-space CG for elasticity against the displacement-form
    Galerkin system assembled densely and solved by LU (GaNi: C^(k - m) wraps
    mod N; Ga on 2N - 1: no wrap)."""
    d = len(N)
    m = d * (d + 1) // 2
    Q = tuple(2 * n - 1 for n in N) if scheme == 1 else N
    A = lame_field(Q, 71 + scheme)
    _, W, _, _ = oracle.Cell(A, N, kind=oracle.ELASTIC, scheme=scheme).solve(np.eye(m), tol=1e-14)
    np.testing.assert_allclose(W, elastic_fourier_galerkin_dense(A, N, scheme, np.eye(m)),
                               rtol=1e-11, atol=1e-11)


@pytest.mark.parametrize("N", [(9, 9), (5, 5, 5)])
def test_elastic_voigt_reuss_bounds(oracle, N):
    """Effective stiffness symmetric, between the Reuss and Voigt averages of
    the Mandel stiffness in the Loewner order; the flux J of unit strains is
    the energy matrix itself (the energy-flux identity at convergence)."""
    d = len(N)
    m = d * (d + 1) // 2
    A = lame_field(N, 81)
    _, W, J, _ = oracle.Cell(A, N, kind=oracle.ELASTIC).solve(np.eye(m), tol=1e-13)
    Cs = np.stack([lame_stiffness(A[0][i], A[1][i], d) for i in np.ndindex(*N)])
    voigt = Cs.mean(axis=0)
    reuss = np.linalg.inv(np.linalg.inv(Cs).mean(axis=0))
    np.testing.assert_allclose(W, W.T, atol=1e-12 * np.abs(W).max())
    assert np.linalg.eigvalsh(voigt - W).min() > -1e-10
    assert np.linalg.eigvalsh(W - reuss).min() > -1e-10
    np.testing.assert_allclose(J, W, rtol=1e-9, atol=1e-9)
