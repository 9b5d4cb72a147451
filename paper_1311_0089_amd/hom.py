"""ctypes binding of ``libhom.so`` (argument marshalling only).

Device memory and streams come from PyTorch: buffers are passed as
``tensor.data_ptr()`` and the current stream as ``hipStream_t``.  Every step
of the solve runs in the library's HIP kernels; nothing here computes.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libhom.so")

GANI, GA = 0, 1
FP64, MIXED = 0, 1
ISO, DIAG, FULLSYM, ELASTIC = 0, 1, 2, 3

EXPORTED_SYMBOLS = [
    "hom_options_default", "hom_create_cell", "hom_solve", "hom_solve_ms", "hom_apply",
    "hom_project",
    "hom_apply_noalloc",
    "hom_profile_iteration", "hom_set_specialized", "hom_autotune", "hom_pass_variants",
    "hom_force_variant", "hom_current_variant", "hom_tune_save",
    "hom_tune_load", "hom_destroy_cell", "hom_status_str", "hom_cell_dims",
    "hom_server_create", "hom_server_submit", "hom_server_poll", "hom_server_times",
    "hom_server_destroy",
]


class HomError(RuntimeError):
    def __init__(self, code: int, what: str):
        msg = lib().hom_status_str(code).decode() if _lib is not None else str(code)
        super().__init__(f"{what}: {msg} ({code})")
        self.code = code


class Options(ctypes.Structure):
    _fields_ = [("scheme", ctypes.c_int), ("prec", ctypes.c_int), ("Y", ctypes.c_double * 3),
                ("max_iter", ctypes.c_int), ("max_outer", ctypes.c_int),
                ("inner_tol", ctypes.c_double), ("check_every", ctypes.c_int),
                ("stream", ctypes.c_void_p), ("a_trig", ctypes.c_int), ("dual", ctypes.c_int)]


class Info(ctypes.Structure):
    _fields_ = [("iters_inner", ctypes.c_int), ("iters_outer", ctypes.c_int),
                ("rel_resid_true", ctypes.c_double), ("rho_A", ctypes.c_double),
                ("seconds", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    """Load libhom.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise ImportError(f"{_LIB_PATH} is missing: build it with "
                              "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = ctypes.CDLL(_LIB_PATH)
        vp, dp, ip = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int
        L.hom_status_str.restype = ctypes.c_char_p
        L.hom_status_str.argtypes = [ip]
        L.hom_options_default.argtypes = [ctypes.POINTER(Options)]
        L.hom_create_cell.argtypes = [ip, ctypes.POINTER(ctypes.c_int32), ip, vp, ip,
                                      ctypes.POINTER(Options), ctypes.POINTER(vp)]
        L.hom_solve.argtypes = [vp, ip, dp, ctypes.c_double, vp, dp, dp, vp, ctypes.POINTER(Info)]
        L.hom_solve_ms.argtypes = [vp, ip, dp, ctypes.c_double, vp, dp, dp, ctypes.POINTER(Info)]
        L.hom_apply.argtypes = [vp, ip, ip, vp, vp]
        L.hom_project.argtypes = [vp, ip, vp, vp]
        L.hom_apply_noalloc.argtypes = [vp, ip, ip, vp, vp]
        L.hom_profile_iteration.argtypes = [vp, ip, ip, ip, dp, dp]
        L.hom_set_specialized.argtypes = [ip]
        L.hom_autotune.argtypes = [vp, ip, ip, ip, dp]
        L.hom_pass_variants.argtypes = [vp, ip, ctypes.POINTER(ctypes.c_int32)]
        L.hom_force_variant.argtypes = [vp, ip, ip, ip]
        L.hom_current_variant.argtypes = [vp, ip, ip, ctypes.POINTER(ctypes.c_int32)]
        L.hom_tune_save.argtypes = [ctypes.c_char_p]
        L.hom_tune_load.argtypes = [ctypes.c_char_p]
        L.hom_destroy_cell.argtypes = [vp]
        L.hom_destroy_cell.restype = None
        L.hom_cell_dims.argtypes = [vp, ctypes.POINTER(ctypes.c_int32),
                                    ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]
        L.hom_server_create.argtypes = [ctypes.c_size_t, ctypes.POINTER(Options), ctypes.POINTER(vp)]
        L.hom_server_submit.argtypes = [vp, vp, ip, dp, ctypes.c_double,
                                        ctypes.POINTER(ctypes.c_uint64)]
        L.hom_server_poll.argtypes = [vp, ctypes.c_uint64, dp, dp, ctypes.POINTER(Info)]
        L.hom_server_times.argtypes = [vp, ctypes.c_uint64, dp]
        L.hom_server_destroy.argtypes = [vp]
        _lib = L
    return _lib


def _check(code: int, what: str, allow=()):
    if code != 0 and code not in allow:
        raise HomError(code, what)
    return code


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _current_stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def set_specialized(enable: bool) -> None:
    """Use (True, default) or bypass (False) the compile-time specialised kernels."""
    _check(lib().hom_set_specialized(1 if enable else 0), "hom_set_specialized")


def tune_save(path: str) -> None:
    _check(lib().hom_tune_save(path.encode()), "hom_tune_save")


def tune_load(path: str) -> bool:
    """Load tuned choices; False if the file is missing or from another GPU."""
    return lib().hom_tune_load(path.encode()) == 0


def make_options(scheme=GANI, prec=FP64, Y=None, max_iter=10000, max_outer=100, inner_tol=1e-3,
                 check_every=16, stream=None, a_trig=False, dual=False) -> Options:
    o = Options()
    lib().hom_options_default(ctypes.byref(o))
    o.scheme, o.prec = scheme, prec
    if Y is not None:
        for a, y in enumerate(Y):
            o.Y[a] = float(y)
    o.max_iter, o.max_outer, o.inner_tol, o.check_every = max_iter, max_outer, inner_tol, check_every
    o.stream = stream
    o.a_trig = 1 if a_trig else 0
    o.dual = 1 if dual else 0
    return o


class Cell:
    """A periodic cell on the current GPU.

    A: coefficient field [nA][Q grid] (numpy float64 on the host, or a torch
    float64 CUDA tensor); N: odd trial sizes; kind: ISO/DIAG/FULLSYM, or
    ELASTIC (A = [lambda, mu], fields as Mandel vectors of d(d+1)/2 components);
    scheme: GANI (A on N) or GA (A on 2N-1); prec: FP64 or MIXED."""

    def __init__(self, A, N, kind=ISO, scheme=GANI, prec=FP64, Y=None, max_iter=10000,
                 max_outer=100, inner_tol=1e-3, check_every=16, a_trig=False, dual=False):
        import torch
        self.N = tuple(int(n) for n in N)
        self.d = len(self.N)
        # field components: d, or the d(d+1)/2 Mandel components of elasticity
        self.nc = self.d * (self.d + 1) // 2 if kind == ELASTIC else self.d
        self.Q = tuple(2 * n - 1 for n in self.N) if scheme == GA else self.N
        self.kind, self.scheme, self.prec = kind, scheme, prec
        self._h = ctypes.c_void_p(None)
        o = make_options(scheme, prec, Y, max_iter, max_outer, inner_tol, check_every,
                         _current_stream(), a_trig, dual)
        Nc = (ctypes.c_int32 * 3)(*(list(self.N) + [1] * (3 - self.d)))
        if isinstance(A, torch.Tensor) and A.is_cuda:
            At = A.to(torch.float64).contiguous()
            ptr, on_dev = ctypes.c_void_p(At.data_ptr()), 1
            keep = At
        else:
            An = np.ascontiguousarray(np.asarray(A, dtype=np.float64))
            ptr, on_dev = ctypes.c_void_p(An.ctypes.data), 0
            keep = An
        _check(lib().hom_create_cell(self.d, Nc, kind, ptr, on_dev, ctypes.byref(o),
                                     ctypes.byref(self._h)), "hom_create_cell")
        del keep

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            lib().hom_destroy_cell(self._h)
            self._h = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, E, tol=1e-8, want_strain=False, strain0=None, allow=()):
        """Solve load cases E [L][d].  Returns dict with W [L][L], J [L][d],
        info and, if requested, the strain field (torch CUDA [L][d][*N])."""
        import torch
        E = np.ascontiguousarray(np.atleast_2d(np.asarray(E, dtype=np.float64)))
        L = E.shape[0]
        W = np.zeros((L, L))
        J = np.zeros((L, self.nc))
        info = Info()
        strain = None
        sp = ctypes.c_void_p(None)
        if want_strain:
            strain = torch.empty((L, self.nc) + self.N, dtype=torch.float64, device="cuda")
            sp = ctypes.c_void_p(strain.data_ptr())
        s0 = ctypes.c_void_p(None)
        if strain0 is not None:
            s0t = strain0.to(torch.float64).contiguous()
            s0 = ctypes.c_void_p(s0t.data_ptr())
        code = lib().hom_solve(self._h, L, _dptr(E), float(tol), sp, _dptr(W), _dptr(J), s0,
                               ctypes.byref(info))
        _check(code, "hom_solve", allow=allow)
        out = {"W": W, "J": J, "info": info.as_dict(), "status": code}
        if want_strain:
            out["strain"] = strain
        return out

    def solve_ms(self, E, tol=1e-8, want_strain=False, allow=()):
        """The Moulinec-Suquet scheme (hom_solve_ms) on load cases E [L][d];
        returns the same dict as solve()."""
        import torch
        E = np.ascontiguousarray(np.atleast_2d(np.asarray(E, dtype=np.float64)))
        L = E.shape[0]
        W = np.zeros((L, L))
        J = np.zeros((L, self.nc))
        info = Info()
        strain = None
        sp = ctypes.c_void_p(None)
        if want_strain:
            strain = torch.empty((L, self.nc) + self.N, dtype=torch.float64, device="cuda")
            sp = ctypes.c_void_p(strain.data_ptr())
        code = lib().hom_solve_ms(self._h, L, _dptr(E), float(tol), sp, _dptr(W), _dptr(J),
                                  ctypes.byref(info))
        _check(code, "hom_solve_ms", allow=allow)
        out = {"W": W, "J": J, "info": info.as_dict(), "status": code}
        if want_strain:
            out["strain"] = strain
        return out

    def apply(self, u, prec=FP64):
        """out = G A G u for real fields u (torch CUDA float64 [L][d][*N])."""
        import torch
        u = u.to(torch.float64).contiguous()
        out = torch.empty_like(u)
        _check(lib().hom_apply(self._h, prec, u.shape[0], ctypes.c_void_p(u.data_ptr()),
                               ctypes.c_void_p(out.data_ptr())), "hom_apply")
        return out

    def apply_noalloc(self, u, out, prec=FP64):
        """hom_apply with the library's fixed scratch as workspace (no device
        allocation inside the call); out: a torch CUDA float64 tensor shaped
        like u, written in place.  Returns the status code."""
        return lib().hom_apply_noalloc(self._h, prec, u.shape[0], ctypes.c_void_p(u.data_ptr()),
                                       ctypes.c_void_p(out.data_ptr()))

    def project(self, u):
        """out = G u (projection onto E_N)."""
        import torch
        u = u.to(torch.float64).contiguous()
        out = torch.empty_like(u)
        _check(lib().hom_project(self._h, u.shape[0], ctypes.c_void_p(u.data_ptr()),
                                 ctypes.c_void_p(out.data_ptr())), "hom_project")
        return out

    def autotune(self, prec=FP64, L=1, reps=10):
        """Pick the fastest kernel variant of every pass (see hom_autotune)."""
        best = np.zeros(5)
        _check(lib().hom_autotune(self._h, prec, L, reps, _dptr(best)), "hom_autotune")
        return best

    def pass_variants(self, prec=FP64):
        """Compile-time variants per pass: [expand, axis-1 inverse, row,
        axis-1 forward, project]."""
        n = (ctypes.c_int32 * 5)()
        _check(lib().hom_pass_variants(self._h, prec, n), "hom_pass_variants")
        return list(n)

    def force_variant(self, pass_index, variant, prec=FP64):
        """Run variant `variant` (-1: generic kernel) of pass `pass_index` for
        every cell of this shape and precision (process-wide)."""
        _check(lib().hom_force_variant(self._h, prec, pass_index, variant), "hom_force_variant")

    def current_variant(self, pass_index, prec=FP64):
        """The variant pass `pass_index` runs now (-1: the generic kernel)."""
        v = ctypes.c_int32(0)
        _check(lib().hom_current_variant(self._h, prec, pass_index, ctypes.byref(v)),
               "hom_current_variant")
        return int(v.value)

    def profile(self, prec=FP64, L=1, reps=20):
        ms = np.zeros(9)
        by = np.zeros(9)
        _check(lib().hom_profile_iteration(self._h, prec, L, reps, _dptr(ms), _dptr(by)),
               "hom_profile_iteration")
        names = ["expand0", "inv1", "row", "fwd1", "project0", "update", "scalars", "iteration",
                 "direction"]
        return {n: {"ms": float(m), "bytes": float(b)} for n, m, b in zip(names, ms, by)}


class Server:
    """Continuous-batching request loop (see hom.h)."""

    def __init__(self, hbm_budget_bytes: int, prec=MIXED, max_iter=10000, inner_tol=1e-3,
                 check_every=16):
        self._h = ctypes.c_void_p(None)
        o = make_options(GANI, prec, None, max_iter, 100, inner_tol, check_every, None)
        _check(lib().hom_server_create(int(hbm_budget_bytes), ctypes.byref(o),
                                       ctypes.byref(self._h)), "hom_server_create")

    def submit(self, cell: Cell, E, tol=1e-6) -> int:
        E = np.ascontiguousarray(np.atleast_2d(np.asarray(E, dtype=np.float64)))
        t = ctypes.c_uint64(0)
        _check(lib().hom_server_submit(self._h, cell.handle, E.shape[0], _dptr(E), float(tol),
                                       ctypes.byref(t)), "hom_server_submit")
        return int(t.value)

    def poll(self, ticket: int, L: int, d: int):
        """None while busy, else dict(W, J, info, status, times)."""
        W = np.zeros((L, L))
        J = np.zeros((L, d))
        info = Info()
        times = np.zeros(3)
        code = lib().hom_server_times(self._h, ticket, _dptr(times))
        if code == -7:
            return None
        code = lib().hom_server_poll(self._h, ticket, _dptr(W), _dptr(J), ctypes.byref(info))
        if code == -7:
            return None
        return {"W": W, "J": J, "info": info.as_dict(), "status": code, "times": times}

    def close(self):
        if self._h:
            _check(lib().hom_server_destroy(self._h), "hom_server_destroy")
            self._h = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
