"""Reference pieces for linear elasticity shared by the oracle pins and the
GPU tests: Mandel vectors, the isotropic Hooke law, seeded Lame fields and
the closed form of a layered medium.  Textbook definitions only (no method
arithmetic of the oracle or the GPU library)."""
import numpy as np

import hom_inputs as hi


# Mandel form: symmetric tensors as d(d+1)/2 vectors in Voigt order with the
# off-diagonal entries times sqrt 2 (so the vector dot product is Z : Z').
def mandel_pairs(d):
    return {2: [(0, 0), (1, 1), (0, 1)], 3: [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]}[d]


def to_mandel(Z, d):
    """(d, d, ...) symmetric tensor -> (m, ...) Mandel vector."""
    return np.stack([Z[a, b] * (1.0 if a == b else np.sqrt(2.0)) for a, b in mandel_pairs(d)])


def from_mandel(z, d):
    Z = np.zeros((d, d) + z.shape[1:], dtype=z.dtype)
    for t, (a, b) in enumerate(mandel_pairs(d)):
        v = z[t] if a == b else z[t] / np.sqrt(2.0)
        Z[a, b] = v
        Z[b, a] = v
    return Z


def lame_stiffness(lam, mu, d):
    """Mandel matrix of lambda tr(eps) I + 2 mu eps (textbook Hooke law)."""
    m = d * (d + 1) // 2
    C = 2.0 * mu * np.eye(m)
    C[:d, :d] += lam
    return C


def lame_field(Q, seed, contrast=20.0):
    """Random Lame fields (lambda, mu) on grid Q: mu in [1, contrast],
    lambda = mu times a factor in [0.2, 2] (positive definite everywhere)."""
    u = hi.uniform(seed, 2 * int(np.prod(Q))).reshape((2,) + tuple(Q))
    mu = 1.0 + (contrast - 1.0) * u[0]
    lam = mu * (0.2 + 1.8 * u[1])
    return np.stack([lam, mu])


def elastic_laminate_W(lam, mu, d):
    """Energy matrix of the unit Mandel strains for layers normal to x_1 with
    grid values lam, mu (closed form of the layered medium: the strains along
    the layers equal the applied ones, the tractions sigma_1b are constant)."""
    m = d * (d + 1) // 2
    W = np.zeros((m, m))
    strains = []
    for I in range(m):
        E = from_mandel(np.eye(m)[I], d)
        eps = np.repeat(E[:, :, None], len(lam), axis=2)
        lam2 = lam + 2.0 * mu
        other = sum(E[b, b] for b in range(1, d))
        s11 = (E[0, 0] + other * np.mean(lam / lam2)) / np.mean(1.0 / lam2)
        eps[0, 0] = (s11 - lam * other) / lam2
        for b in range(1, d):
            s1b = 2.0 * E[0, b] / np.mean(1.0 / mu)
            eps[0, b] = eps[b, 0] = s1b / (2.0 * mu)
        strains.append(to_mandel(eps, d))
    for I in range(m):
        for J in range(m):
            W[I, J] = np.mean([strains[I][:, p] @ lame_stiffness(lam[p], mu[p], d) @ strains[J][:, p]
                               for p in range(len(lam))])
    return W
