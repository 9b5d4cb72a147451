"""Seeded generators: determinism, the published SplitMix64 sequence, and the
fast inclusion / majority-filter code against their direct definitions."""
import numpy as np

import hom_inputs as hi


def test_splitmix64_reference_values():
    # first outputs for seed 0 of the published SplitMix64 (Vigna's splitmix64.c)
    z = hi.splitmix64(0, 3)
    assert [int(v) for v in z] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_uniform_and_normal_statistics():
    u = hi.uniform(1, 200_000)
    assert 0.0 <= u.min() and u.max() < 1.0 and abs(u.mean() - 0.5) < 5e-3
    g = hi.normal(2, 200_000)
    assert abs(g.mean()) < 1e-2 and abs(g.std() - 1.0) < 1e-2


def _inclusions_direct(N, count, r, a_in, seed):
    d = len(N)
    C = hi.rsa_centres(d, count, r, seed)
    X = hi.mesh(N)
    inside = np.zeros(N, bool)
    for c in C:
        dist2 = np.zeros(N)
        for a in range(d):
            dx = X[a] - (c[a] - 0.5)
            dx -= np.round(dx)
            dist2 += dx * dx
        inside |= dist2 < r * r
    return np.where(inside, a_in, 1.0)


def _majority_direct(N, p, passes, seed):
    ph = (hi.uniform(seed, int(np.prod(N))) < p).reshape(N).astype(np.int32)
    k = 3 ** len(N)
    for _ in range(passes):
        s = np.zeros(N, np.int32)
        for sh in np.ndindex(*(3,) * len(N)):
            s += np.roll(ph, tuple(int(t) - 1 for t in sh), axis=tuple(range(len(N))))
        ph = (2 * s > k).astype(np.int32)
    return ph


def test_fast_generators_equal_direct_definitions():
    for N in [(63, 63), (31, 33, 35)]:
        assert np.array_equal(hi.inclusions(N, 12, 0.06, 5.0, seed=7),
                              _inclusions_direct(N, 12, 0.06, 5.0, 7))
        assert np.array_equal(hi.bernoulli_majority(N, 0.4, 3, 2.0, 1.0, seed=3) > 1.5,
                              _majority_direct(N, 0.4, 3, 3) == 1)


def test_rsa_non_overlapping_and_square_fraction():
    C = hi.rsa_centres(3, 60, 0.06, 3)
    for i in range(len(C)):
        for j in range(i):
            dd = C[i] - C[j]
            dd -= np.round(dd)
            assert np.dot(dd, dd) >= (0.12) ** 2
    w = hi.cfg1_square()
    assert abs(w.info["vf"] - 49 / 225) < 1e-15


def test_fourier_coefficients_of_inclusions_by_quadrature():
    """The analytic Fourier coefficients used for exact integration (interval,
    disc, ball) against a midpoint-rule integral of the indicator on a fine
    grid: A^(k) = integral over the unit cell of chi exp(-2 pi i k.x)."""
    n = 1200
    x = (np.arange(n) + 0.5) / n - 0.5
    chi = (np.abs(x) < 0.2).astype(float)
    for k in (0, 1, 3, 7):
        num = np.sum(chi * np.exp(-2j * np.pi * k * x)) / n
        assert abs(num - hi._interval_coef(k, 0.2)) < 2e-3
    X, Yg = np.meshgrid(x, x, indexing="ij")
    disc = (X ** 2 + Yg ** 2 < 0.3 ** 2).astype(float)
    for k in ((0, 0), (1, 0), (2, 1), (3, 4)):
        num = np.sum(disc * np.exp(-2j * np.pi * (k[0] * X + k[1] * Yg))) / n ** 2
        ref = hi.ball_coef(np.hypot(*k), 0.3, 2)
        assert abs(num - ref) < 2e-3 * np.pi * 0.09
    m = 160
    x3 = (np.arange(m) + 0.5) / m - 0.5
    X3 = np.meshgrid(x3, x3, x3, indexing="ij")
    ball = (X3[0] ** 2 + X3[1] ** 2 + X3[2] ** 2 < 0.25 ** 2).astype(float)
    for k in ((0, 0, 0), (1, 0, 0), (1, 1, 2)):
        num = np.sum(ball * np.exp(-2j * np.pi * sum(a * b for a, b in zip(k, X3)))) / m ** 3
        ref = hi.ball_coef(np.sqrt(sum(a * a for a in k)), 0.25, 3)
        assert abs(num - ref) < 1e-2 * 4 / 3 * np.pi * 0.25 ** 3


def test_trig_samples_are_the_truncated_series():
    """Samples on M = 2N-1 of the truncated series: their grid mean is the
    exact volume average, their DFT returns the analytic coefficients, and
    the series converges to the indicator at the centre of an inclusion."""
    N = (9, 7)
    A = hi.square_inclusion_trig(N, 0.25, 10.0, 1.0)
    assert A.shape == (17, 13)
    assert abs(A.mean() - (1.0 + 9.0 * 0.25)) < 1e-13
    Ahat = np.fft.fftn(A) / A.size
    k0, k1 = hi.signed_index(17), hi.signed_index(13)
    ref = 9.0 * np.outer(hi._interval_coef(k0, 0.25), hi._interval_coef(k1, 0.25))
    ref[0, 0] += 1.0
    np.testing.assert_allclose(Ahat, ref, atol=1e-13)
    vals = [hi.square_inclusion_trig((n, n), 0.25, 2.0, 1.0)[0, 0] for n in (9, 33, 129)]
    assert abs(vals[-1] - 2.0) < abs(vals[0] - 2.0) and abs(vals[-1] - 2.0) < 0.05
    S = hi.inclusions_trig((9, 9, 9), 1, 0.2, 5.0, 1.0, centres=[[0.5, 0.5, 0.5]])
    assert abs(S.mean() - (1.0 + 4.0 * 4.0 / 3.0 * np.pi * 0.2 ** 3)) < 1e-13
    # a shifted centre moves the field: the sample at the new centre is the old
    # centre's value (grid-aligned shift of 2 cells of the 17-point grid)
    S2 = hi.inclusions_trig((9, 9, 9), 1, 0.2, 5.0, 1.0, centres=[[0.5 + 2 / 17, 0.5, 0.5]])
    np.testing.assert_allclose(S2[2], S[0], atol=1e-12)
