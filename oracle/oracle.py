"""ctypes binding of the FP64 CPU oracle (``hom_oracle.c``).

TEST INFRASTRUCTURE ONLY.  The test suite, the smoke entry point and the
benchmark's CPU-baseline leg are the only callers; the GPU library never
imports this module and this module never imports the GPU library.

Array conventions follow ``hom_oracle.h``: real vector fields are numpy
float64 arrays of shape ``(d, *N)`` in FFT order; the coefficient field has
shape ``(nA, *Q)``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hom_oracle.c")
_LIB = os.environ.get("HOM_ORACLE_LIB") or os.path.join(_HERE, "libhom_oracle.so")

ISO, DIAG, FULLSYM, ELASTIC = 0, 1, 2, 3
GANI, GA = 0, 1
_ERR = {0: "ok", -1: "invalid argument", -2: "imaginary part not negligible",
        -3: "out of memory", -4: "not converged", -5: "CG breakdown"}


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {_ERR.get(code, code)}")
        self.code = code


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C99 + OpenMP, FP64)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                               "-D_DEFAULT_SOURCE", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Cell(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int), ("scheme", ctypes.c_int), ("kind", ctypes.c_int),
                ("dual", ctypes.c_int), ("N", ctypes.c_long * 3), ("Q", ctypes.c_long * 3),
                ("Y", ctypes.c_double * 3), ("A", ctypes.POINTER(ctypes.c_double))]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        dp = P(ctypes.c_double)
        cp = P(_Cell)
        L.hor_dft_axis.argtypes = [ctypes.c_int, P(ctypes.c_long), ctypes.c_int, ctypes.c_int, dp]
        L.hor_dft_all.argtypes = [ctypes.c_int, P(ctypes.c_long), ctypes.c_int, dp]
        L.hor_apply_G.argtypes = [cp, dp, dp]
        L.hor_apply_GA.argtypes = [cp, dp, dp]
        L.hor_cg.argtypes = [cp, dp, ctypes.c_double, ctypes.c_int, ctypes.c_int, dp,
                             P(ctypes.c_int), dp, dp]
        L.hor_cg_lsd.argtypes = [cp, dp, ctypes.c_double, ctypes.c_double, ctypes.c_int, dp,
                                 P(ctypes.c_int)]
        L.hor_ms.argtypes = [cp, dp, ctypes.c_double, ctypes.c_double, ctypes.c_int, dp,
                             P(ctypes.c_int)]
        L.hor_homogenized.argtypes = [cp, ctypes.c_int, dp, dp, dp, dp]
        L.hor_strain_on_Q.argtypes = [cp, dp, dp, dp]
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _chk(code: int, what: str, allow=()):
    if code != 0 and code not in allow:
        raise OracleError(code, what)
    return code


def n_coeff(kind: int, d: int) -> int:
    return {ISO: 1, DIAG: d, FULLSYM: d * (d + 1) // 2, ELASTIC: 2}[kind]


def n_comp(kind: int, d: int) -> int:
    """Field components: d, or d(d+1)/2 Mandel components for elasticity."""
    return d * (d + 1) // 2 if kind == ELASTIC else d


class Cell:
    """A periodic cell: trial grid N (odd), coefficient field A on the
    quadrature grid Q (N for GaNi, 2N-1 for Ga) and half-lengths Y."""

    def __init__(self, A: np.ndarray, N, kind: int = ISO, scheme: int = GANI, Y=None,
                 dual: bool = False):
        N = tuple(int(n) for n in N)
        d = len(N)
        Q = tuple(2 * n - 1 for n in N) if scheme == GA else N
        A = np.ascontiguousarray(A, dtype=np.float64)
        if A.shape == Q and kind == ISO:
            A = A.reshape((1,) + Q)
        if A.shape != (n_coeff(kind, d),) + Q:
            raise ValueError(f"A has shape {A.shape}, expected {(n_coeff(kind, d),) + Q}")
        self.A, self.N, self.Q, self.d, self.kind, self.scheme = A, N, Q, d, kind, scheme
        self.nc = n_comp(kind, d)
        self.Y = tuple(Y) if Y is not None else (0.5,) * d
        c = _Cell()
        c.d, c.scheme, c.kind = d, scheme, kind
        c.dual = 1 if dual else 0
        for a in range(3):
            c.N[a] = N[a] if a < d else 1
            c.Q[a] = Q[a] if a < d else 1
            c.Y[a] = self.Y[a] if a < d else 1.0
        c.A = _dp(self.A)
        self._c = c

    # -- operators ------------------------------------------------------
    def _field(self, u):
        u = np.ascontiguousarray(u, dtype=np.float64)
        if u.shape != (self.nc,) + self.N:
            raise ValueError(f"field shape {u.shape} != {(self.nc,) + self.N}")
        return u

    def apply_G(self, u):
        u = self._field(u)
        out = np.empty_like(u)
        _chk(lib().hor_apply_G(ctypes.byref(self._c), _dp(u), _dp(out)), "apply_G")
        return out

    def apply_GA(self, u):
        u = self._field(u)
        out = np.empty_like(u)
        _chk(lib().hor_apply_GA(ctypes.byref(self._c), _dp(u), _dp(out)), "apply_GA")
        return out

    # -- solvers ----------------------------------------------------------
    def cg(self, E, tol=1e-8, max_iter=10000, x0=None, history=False, allow_notconv=False):
        """CG on G A x = -G A E (x0 = 0 unless given).  Returns
        (x, iters, true relative residual[, history])."""
        E = np.ascontiguousarray(E, dtype=np.float64).reshape(self.nc)
        x = np.zeros((self.nc,) + self.N) if x0 is None else self._field(x0).copy()
        it = ctypes.c_int(0)
        rr = ctypes.c_double(0.0)
        hist = np.zeros(max_iter + 1)
        code = lib().hor_cg(ctypes.byref(self._c), _dp(E), tol, max_iter, int(x0 is not None),
                            _dp(x), ctypes.byref(it), ctypes.byref(rr), _dp(hist))
        _chk(code, "cg", allow=(-4,) if allow_notconv else ())
        if history:
            return x, it.value, rr.value, hist[: it.value + 1]
        return x, it.value, rr.value

    def cg_lsd(self, E, lam, tol=1e-12, max_iter=10000):
        E = np.ascontiguousarray(E, dtype=np.float64).reshape(self.nc)
        e = np.empty((self.nc,) + self.N)
        it = ctypes.c_int(0)
        _chk(lib().hor_cg_lsd(ctypes.byref(self._c), _dp(E), lam, tol, max_iter, _dp(e),
                              ctypes.byref(it)), "cg_lsd")
        return e, it.value

    def ms(self, E, lam, tol=1e-12, max_iter=100000):
        E = np.ascontiguousarray(E, dtype=np.float64).reshape(self.nc)
        e = np.empty((self.nc,) + self.N)
        it = ctypes.c_int(0)
        _chk(lib().hor_ms(ctypes.byref(self._c), _dp(E), lam, tol, max_iter, _dp(e),
                          ctypes.byref(it)), "ms")
        return e, it.value

    def homogenized(self, E, x):
        """W_lm = <e_l . A e_m>_Q and J_l = <A e_l>_Q for load cases E [L][d]
        and fluctuations x [L][d][N]."""
        E = np.ascontiguousarray(E, dtype=np.float64).reshape(-1, self.nc)
        L = E.shape[0]
        x = np.ascontiguousarray(x, dtype=np.float64).reshape((L, self.nc) + self.N)
        W = np.empty((L, L))
        J = np.empty((L, self.nc))
        _chk(lib().hor_homogenized(ctypes.byref(self._c), L, _dp(E), _dp(x), _dp(W), _dp(J)),
             "homogenized")
        return W, J

    def strain_on_Q(self, E, x):
        E = np.ascontiguousarray(E, dtype=np.float64).reshape(self.nc)
        x = self._field(x)
        out = np.empty((self.nc,) + self.Q)
        _chk(lib().hor_strain_on_Q(ctypes.byref(self._c), _dp(E), _dp(x), _dp(out)),
             "strain_on_Q")
        return out

    def solve(self, E, tol=1e-8, max_iter=10000):
        """Solve every load case of E [L][d] (elasticity: [L][d(d+1)/2] Mandel
        strains); returns (x [L][nc][N], W, J, iters)."""
        E = np.ascontiguousarray(E, dtype=np.float64).reshape(-1, self.nc)
        xs, its = [], []
        for El in E:
            x, it, _ = self.cg(El, tol=tol, max_iter=max_iter)
            xs.append(x)
            its.append(it)
        x = np.stack(xs)
        W, J = self.homogenized(E, x)
        return x, W, J, its


def dft_axis(z: np.ndarray, axis: int, sign: int) -> np.ndarray:
    """Naive DFT of a complex array along one axis (sign -1: forward with 1/n)."""
    z = np.ascontiguousarray(z, dtype=np.complex128).copy()
    n = (ctypes.c_long * z.ndim)(*z.shape)
    _chk(lib().hor_dft_axis(z.ndim, n, axis, sign, _dp(z.view(np.float64))), "dft_axis")
    return z


def dft_all(z: np.ndarray, sign: int) -> np.ndarray:
    z = np.ascontiguousarray(z, dtype=np.complex128).copy()
    n = (ctypes.c_long * z.ndim)(*z.shape)
    _chk(lib().hor_dft_all(z.ndim, n, sign, _dp(z.view(np.float64))), "dft_all")
    return z
