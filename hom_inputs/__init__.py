"""Seeded synthetic inputs for the periodic cell problem.

This module is shared by the tests, the benchmark, the CPU oracle's callers
and the GPU library's callers.  It holds generators only: random numbers,
geometry and coefficient fields.  None of the homogenization arithmetic (DFT,
projection, solver, quadrature) lives here.

Random numbers come from SplitMix64 (Steele, Lea & Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014): state_i = seed + i * gamma,
output = mix(state_i).  Uniforms are (z >> 11) * 2**-53; normals use the
Box-Muller transform with u1 in (0, 1].  Grid draws are made in FFT-order,
row-major over the grid.

Grids follow the paper's convention: on a cell prod [-Y_a, Y_a] with N_a odd
points per axis, storage index i holds x = k h with k = i if i <= (N-1)/2 else
i - N and h = 2 Y / N, so the origin is index 0.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, n: int, offset: int = 0) -> np.ndarray:
    """n outputs of SplitMix64 started from ``seed`` (outputs offset+1 .. offset+n)."""
    with np.errstate(over="ignore"):
        i = np.arange(offset + 1, offset + n + 1, dtype=np.uint64)
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + i * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def splitmix_one(seed: int, i: int) -> int:
    """The i-th output (i >= 1) of SplitMix64 from ``seed``, as a Python int."""
    return int(splitmix64(seed, 1, offset=i - 1)[0])


def uniform(seed: int, n: int, offset: int = 0) -> np.ndarray:
    """n uniforms in [0, 1) with 53 random bits."""
    return (splitmix64(seed, n, offset) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53


def normal(seed: int, n: int) -> np.ndarray:
    """n standard normals by Box-Muller from consecutive uniform pairs."""
    m = (n + 1) // 2
    u = uniform(seed, 2 * m).reshape(m, 2)
    u1 = 1.0 - u[:, 0]              # (0, 1]
    rad = np.sqrt(-2.0 * np.log(u1))
    th = 2.0 * np.pi * u[:, 1]
    z = np.stack([rad * np.cos(th), rad * np.sin(th)], axis=1).reshape(-1)
    return z[:n]


# --------------------------------------------------------------------------
# grids
# --------------------------------------------------------------------------

def signed_index(n: int) -> np.ndarray:
    """Signed index k of each storage position on an axis of length n."""
    i = np.arange(n)
    return np.where(i <= (n - 1) // 2, i, i - n)


def coords(N, Y=None):
    """Grid coordinates x_a = k h_a (open grid, origin at index 0), one 1-D
    array per axis."""
    d = len(N)
    Y = (0.5,) * d if Y is None else Y
    return [signed_index(n) * (2.0 * y / n) for n, y in zip(N, Y)]


def mesh(N, Y=None):
    return np.meshgrid(*coords(N, Y), indexing="ij")


# --------------------------------------------------------------------------
# microstructures
# --------------------------------------------------------------------------

def square_inclusion(N, half_width=0.25, a_in=10.0, a_out=1.0, Y=None):
    """Centred square (cube) inclusion: a_in where max_a |x_a| < half_width."""
    X = mesh(N, Y)
    inside = np.ones(tuple(N), dtype=bool)
    for x in X:
        inside &= np.abs(x) < half_width
    return np.where(inside, a_in, a_out).astype(np.float64)


def _neighbour_sum(ph):
    """Periodic sum over the 3^d Moore neighbourhood (centre included)."""
    try:
        from scipy.ndimage import convolve
        return convolve(ph, np.ones((3,) * ph.ndim, dtype=ph.dtype), mode="wrap")
    except ImportError:  # pragma: no cover - scipy is part of the image
        s = np.zeros_like(ph)
        for shift in np.ndindex(*(3,) * ph.ndim):
            s += np.roll(ph, tuple(int(t) - 1 for t in shift), axis=tuple(range(ph.ndim)))
        return s


def bernoulli_majority(N, p=0.4, passes=3, a1=100.0, a0=1.0, seed=2):
    """Two-phase pixel field: phase 1 with probability p per pixel (uniform < p,
    FFT-order row-major draws), then ``passes`` synchronous periodic 3^d Moore
    majority votes (phase 1 iff more than half of the 3^d cells, centre
    included, are phase 1).  Returns the conductivity field."""
    N = tuple(N)
    ph = (uniform(seed, int(np.prod(N))) < p).reshape(N).astype(np.int32)
    k = 3 ** len(N)
    for _ in range(passes):
        ph = (2 * _neighbour_sum(ph) > k).astype(np.int32)
    return np.where(ph == 1, a1, a0).astype(np.float64)


def rsa_centres(d, count, r, seed, max_draws=10_000_000):
    """Random sequential addition: uniform centres in [0,1)^d, a candidate is
    accepted when its periodic minimum-image distance to every accepted centre
    is >= 2r; stops at ``count`` centres."""
    centres = []
    off = 0
    batch = 4096
    draws = 0
    while len(centres) < count:
        u = uniform(seed, batch * d, offset=off).reshape(batch, d)
        off += batch * d
        for c in u:
            draws += 1
            if draws > max_draws:
                raise RuntimeError("RSA did not place all inclusions")
            ok = True
            for q in centres:
                dd = c - q
                dd -= np.round(dd)
                if float(np.dot(dd, dd)) < (2 * r) ** 2:
                    ok = False
                    break
            if ok:
                centres.append(c.copy())
                if len(centres) == count:
                    break
    return np.array(centres)


def inclusions(N, count, r, a_in, a_out=1.0, seed=3):
    """Non-overlapping discs/spheres of radius r (cell of unit size), centres
    by RSA; a grid point is inside when its minimum-image distance to a centre
    is < r.  Only the grid points in each centre's bounding box are tested."""
    N = tuple(N)
    d = len(N)
    C = rsa_centres(d, count, r, seed)
    xs = coords(N)
    inside = np.zeros(N, dtype=bool)
    for c in C:
        idx, dxs = [], []
        for a in range(d):
            n = N[a]
            h = 1.0 / n
            cx = c[a] - 0.5                       # centres drawn in [0,1) -> cell [-1/2, 1/2)
            k = np.arange(int(np.floor((cx - r) / h)) - 1, int(np.ceil((cx + r) / h)) + 2)
            i = np.unique(np.mod(k, n))
            dx = xs[a][i] - cx
            dx -= np.round(dx)
            idx.append(i)
            dxs.append(dx)
        dist2 = np.zeros([len(i) for i in idx])
        for a in range(d):
            shape = [1] * d
            shape[a] = -1
            dist2 = dist2 + (dxs[a] * dxs[a]).reshape(shape)
        sub = inside[np.ix_(*idx)]
        inside[np.ix_(*idx)] = sub | (dist2 < r * r)
    return np.where(inside, a_in, a_out).astype(np.float64)


# --------------------------------------------------------------------------
# coefficients given by their Fourier coefficients: samples on the doubled
# grid of the truncated series (unit cell [-1/2, 1/2)^d, A(x) = sum_k A^(k)
# exp(2 pi i k.x), A^(k) = integral of A exp(-2 pi i k.x))
# --------------------------------------------------------------------------

def trig_samples(M, coef):
    """Samples on the grid M (FFT order) of the trigonometric polynomial whose
    coefficients coef (array over Z_M, FFT order) are given."""
    M = tuple(M)
    return (np.fft.ifftn(coef) * float(np.prod(M))).real


def _interval_coef(k, half_width):
    """Fourier coefficients of the indicator of [-w, w] on the unit period."""
    k = np.asarray(k, dtype=np.float64)
    safe = np.where(k == 0, 1.0, k)
    return np.where(k == 0, 2.0 * half_width, np.sin(2.0 * np.pi * safe * half_width) / (np.pi * safe))


def laminate_step_trig(N, width, a_in, a_out=1.0):
    """Layer |x_1| < width/2 of a_in in a_out, as samples of its truncated
    Fourier series on M = 2N-1 (volume fraction width exactly)."""
    M = tuple(2 * n - 1 for n in N)
    coef = np.zeros(M, dtype=complex)
    k0 = signed_index(M[0])
    line = (a_in - a_out) * _interval_coef(k0, 0.5 * width)
    line[0] += a_out
    coef[(slice(None),) + (0,) * (len(M) - 1)] = line
    return trig_samples(M, coef)


def square_inclusion_trig(N, half_width=0.25, a_in=10.0, a_out=1.0):
    """Centred square / cube max |x_a| < half_width of a_in in a_out, as
    samples of its truncated Fourier series on M = 2N-1 (a product of
    sinc-type factors; volume fraction (2 half_width)^d exactly)."""
    M = tuple(2 * n - 1 for n in N)
    chi = np.ones(M)
    for a, m in enumerate(M):
        shape = [1] * len(M)
        shape[a] = m
        chi = chi * _interval_coef(signed_index(m), half_width).reshape(shape)
    coef = (a_in - a_out) * chi.astype(complex)
    coef[(0,) * len(M)] += a_out
    return trig_samples(M, coef)


def ball_coef(q, r, d):
    """Fourier coefficient of the indicator of a disc (d = 2) or ball (d = 3)
    of radius r at the origin, at wavenumber magnitude q (cycles per cell)."""
    from scipy.special import j1
    q = np.asarray(q, dtype=np.float64)
    z = 2.0 * np.pi * q * r
    zs = np.where(z == 0, 1.0, z)
    if d == 2:
        return np.where(z == 0, np.pi * r * r, 2.0 * np.pi * r * r * j1(zs) / zs)
    return np.where(z == 0, 4.0 * np.pi * r ** 3 / 3.0,
                    4.0 * np.pi * r ** 3 * (np.sin(zs) - zs * np.cos(zs)) / zs ** 3)


def inclusions_trig(N, count, r, a_in, a_out=1.0, seed=3, centres=None):
    """The discs / spheres of ``inclusions`` (same RSA centres) as samples of
    the truncated Fourier series on M = 2N-1: A^(k) = a_out [k = 0] +
    (a_in - a_out) B^(|k|) sum_c exp(-2 pi i k.c)."""
    N = tuple(N)
    d = len(N)
    M = tuple(2 * n - 1 for n in N)
    C = rsa_centres(d, count, r, seed) if centres is None else np.asarray(centres)
    ks = [signed_index(m).astype(np.float64) for m in M]
    phase = np.zeros(M, dtype=complex)
    for c in C:
        term = np.ones((1,) * d, dtype=complex)
        for a in range(d):
            shape = [1] * d
            shape[a] = M[a]
            term = term * np.exp(-2j * np.pi * ks[a] * (c[a] - 0.5)).reshape(shape)
        phase += term
    q2 = np.zeros(M)
    for a in range(d):
        shape = [1] * d
        shape[a] = M[a]
        q2 = q2 + (ks[a] ** 2).reshape(shape)
    coef = (a_in - a_out) * ball_coef(np.sqrt(q2), r, d) * phase
    coef[(0,) * d] += a_out
    return trig_samples(M, coef)


def gaussian_field(M, ell=0.1, sigma=1.5, seed=4):
    """Stationary Gaussian field on the periodic grid M by circulant embedding:
    lambda = DFT of the periodised covariance sigma^2 exp(-|r|^2 / (2 ell^2))
    (minimum-image r), negative eigenvalues clipped to 0, g = IDFT(sqrt(lambda)
    DFT(w)) for white N(0,1) noise w; the sample mean is removed."""
    M = tuple(M)
    X = mesh(M)
    r2 = np.zeros(M)
    for x in X:
        r2 += x * x                 # coordinates are already minimum-image in [-1/2, 1/2)
    cov = sigma ** 2 * np.exp(-r2 / (2 * ell * ell))
    lam = np.fft.fftn(cov).real
    lam = np.maximum(lam, 0.0)
    w = normal(seed, int(np.prod(M))).reshape(M)
    g = np.fft.ifftn(np.sqrt(lam) * np.fft.fftn(w)).real
    return g - g.mean()


def lognormal_diag(M, factors=(1.0, 2.0, 0.5), ell=0.1, sigma=1.5, seed=4):
    """Diagonal coefficient field A = exp(g) diag(factors) on grid M:
    returns (nA=d, *M)."""
    g = gaussian_field(M, ell, sigma, seed)
    eg = np.exp(g)
    return np.stack([f * eg for f in factors])


def laminate(N, values_along_axis0):
    """Isotropic laminate a(x_1): values given per grid index along axis 0."""
    N = tuple(N)
    v = np.asarray(values_along_axis0, dtype=np.float64)
    assert v.shape == (N[0],)
    return np.broadcast_to(v.reshape((N[0],) + (1,) * (len(N) - 1)), N).copy()


def random_spd_field(N, kind, seed, contrast=10.0):
    """Random SPD coefficient field of the given kind (0 iso, 1 diag,
    2 full symmetric) with eigenvalues in [1, contrast]."""
    N = tuple(N)
    d = len(N)
    n = int(np.prod(N))
    if kind == 0:
        return (1.0 + (contrast - 1.0) * uniform(seed, n)).reshape(N)
    if kind == 1:
        return (1.0 + (contrast - 1.0) * uniform(seed, d * n)).reshape((d,) + N)
    # full symmetric: Q diag(l) Q^T with Q from a random rotation per point
    lam = 1.0 + (contrast - 1.0) * uniform(seed, d * n).reshape(n, d)
    g = normal(seed + 1, d * d * n).reshape(n, d, d)
    Qm, _ = np.linalg.qr(g)
    A = np.einsum("pab,pb,pcb->pac", Qm, lam, Qm)
    if d == 1:
        idx = [(0, 0)]
    elif d == 2:
        idx = [(0, 0), (1, 1), (0, 1)]
    else:
        idx = [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]
    return np.stack([A[:, a, b].reshape(N) for a, b in idx])


# --------------------------------------------------------------------------
# named workloads (the configurations the library is measured on)
# --------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    d: int
    N: tuple
    scheme: int            # 0 GaNi, 1 Ga
    kind: int              # 0 iso, 1 diag, 2 full symmetric, 3 isotropic elasticity
    A: np.ndarray          # (nA, *Q) or Q for iso
    E: np.ndarray          # (L, d)
    tol: float
    info: dict = field(default_factory=dict)


def cfg1_square():
    """2-D, N = 15^2, centred square of conductivity 10 in a matrix of 1,
    E = (1, 0), tol 1e-8 (grid samples |x_a| < 0.25 give 7x7 pixels)."""
    N = (15, 15)
    A = square_inclusion(N, 0.25, 10.0, 1.0)
    return Workload("square-15x15-fp64", 2, N, 0, 0, A, np.array([[1.0, 0.0]]), 1e-8,
                    {"vf": float((A > 1).mean()), "contrast": 10.0})


def cfg2_pixels(N=(1023, 1023), seed=2):
    """2-D two-phase pixels: Bernoulli(0.4) + 3 majority passes, phases 100 / 1,
    E = e1, e2, tol 1e-6."""
    A = bernoulli_majority(N, 0.4, 3, 100.0, 1.0, seed)
    return Workload(f"pixels-{N[0]}x{N[1]}", 2, tuple(N), 0, 0, A, np.eye(2), 1e-6,
                    {"vf": float((A > 1).mean()), "contrast": 100.0, "seed": seed})


def cfg3_spheres(N=(255, 255, 255), count=60, r=0.06, seed=3):
    """3-D, 60 RSA spheres of radius 0.06, conductivity 1e3 / 1, E = e1..e3."""
    A = inclusions(N, count, r, 1e3, 1.0, seed)
    return Workload(f"spheres-{N[0]}^3", 3, tuple(N), 0, 0, A, np.eye(3), 1e-6,
                    {"vf": float((A > 1).mean()), "contrast": 1e3, "seed": seed})


def elastic_spheres(N=(255, 255, 255), count=60, r=0.06, seed=3, contrast=100.0):
    """3-D linear elasticity: the 60 spheres of the sphere workload as stiff
    isotropic inclusions (Lame lambda = mu = contrast) in a matrix with
    lambda = mu = 1 (Poisson ratio 1/4); A = [lambda, mu]; the six unit Mandel
    strains as load cases."""
    inside = inclusions(N, count, r, 2.0, 1.0, seed) > 1.0
    lam = np.where(inside, contrast, 1.0)
    A = np.stack([lam, lam.copy()])
    return Workload(f"elastic-spheres-{N[0]}^3", 3, tuple(N), 0, 3, A, np.eye(6), 1e-6,
                    {"vf": float(inside.mean()), "contrast": contrast, "seed": seed})


def cfg4_lognormal(N=(127, 127, 127), seed=4):
    """3-D Ga: trial grid N, lognormal diagonal coefficient on the 2N-1 grid."""
    M = tuple(2 * n - 1 for n in N)
    A = lognormal_diag(M, (1.0, 2.0, 0.5), 0.1, 1.5, seed)
    lo = float(A.min(axis=0).min())
    hi = float(A.max(axis=0).max())
    return Workload(f"lognormal-Ga-{N[0]}^3-on-{M[0]}^3", 3, tuple(N), 1, 1, A, np.eye(3), 1e-6,
                    {"contrast": hi / lo, "seed": seed})


@dataclass
class Request:
    idx: int
    arrival: float
    d: int
    N: tuple
    E: np.ndarray
    tol: float
    contrast: float
    kind_micro: str          # "inclusions" or "pixels"
    seed: int
    count: int               # inclusions: number of discs/spheres
    geometry_seed: int       # seed of the geometry actually drawn (see serving_stream)

    def field(self) -> np.ndarray:
        """Isotropic two-phase conductivity field of this request."""
        if self.kind_micro == "inclusions":
            return inclusions(self.N, self.count, 0.06, self.contrast, 1.0, seed=self.geometry_seed)
        return bernoulli_majority(self.N, 0.4, 3, self.contrast, 1.0, seed=self.geometry_seed)


def serving_stream(n_requests=10_000, rate=500.0, seed=5, sizes2=(63, 127, 255),
                   sizes3=(31, 63, 127), tol=1e-6, geometry_pool=0):
    """Seeded request stream: Poisson arrivals (mean rate), d in {2,3} with
    p = 1/2, N uniform from the size list, half RSA inclusions (count U{5..40}
    in 2-D, U{10..60} in 3-D, r = 0.06), half Bernoulli pixels (p = 0.4, 3
    majority passes), contrast 10^(1+3u), L = 1 + floor(u d) load cases
    e_1..e_L.  Request i draws from seed_i = splitmix(seed, i).  With
    geometry_pool > 0 the geometry (not the contrast) is taken from a pool of
    that many seeds per (d, N, type), so fields can be cached."""
    t = 0.0
    out = []
    head = uniform(seed, n_requests)
    for i in range(n_requests):
        si = splitmix_one(seed, i + 1)
        u = uniform(si, 8)
        t += -math.log(1.0 - head[i]) / rate
        d = 2 if u[0] < 0.5 else 3
        sizes = sizes2 if d == 2 else sizes3
        n = sizes[min(int(u[1] * len(sizes)), len(sizes) - 1)]
        contrast = 10.0 ** (1.0 + 3.0 * u[2])
        L = 1 + min(int(u[3] * d), d - 1)
        incl = u[4] < 0.5
        lo, hi = (5, 40) if d == 2 else (10, 60)
        cnt = lo + min(int(u[5] * (hi - lo + 1)), hi - lo)
        gseed = si if geometry_pool <= 0 else splitmix_one(seed + 1000 * d + n,
                                                            1 + int(u[6] * geometry_pool))
        out.append(Request(i, t, d, (n,) * d, np.eye(d)[:L], tol, contrast,
                           "inclusions" if incl else "pixels", si, cnt, gseed))
    return out
