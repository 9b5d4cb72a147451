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
