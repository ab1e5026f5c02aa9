"""ctypes front-end of the FP64 CPU oracle (liboracle.so, built from oracle.c).

TEST INFRASTRUCTURE: only the tests, the package smoke check and the CPU-baseline leg of
the benchmark use this package.  It imports nothing from the HIP library and the HIP
library imports nothing from it.

Every field is a float64 numpy array of shape (3, nz, ny, nx) (x fastest); a grid is any
object with attributes n (nx, ny, nz), h (hx, hy, hz) and bc (0 line-tied, 1 periodic).
"""
from __future__ import annotations

import contextlib
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("ORACLE_LIB", os.path.join(HERE, "liboracle.so"))

OK, E_ARG, E_FOLD, E_DT, E_NAN, E_MEM = 0, -1, -3, -4, -5, -7

_lib = None
_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_zp = np.ctypeslib.ndpointer(dtype=np.complex128, flags="C_CONTIGUOUS")


def lib():
    """Load liboracle.so, building it first if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        from . import build as _b
        _b.build()
    L = C.CDLL(LIB_PATH)
    i3 = C.POINTER(C.c_int)
    d3 = C.POINTER(C.c_double)
    L.orc_fields.argtypes = [i3, d3, i3, C.c_double, _dp, _dp, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    L.orc_diagnostics.argtypes = [i3, d3, i3, C.c_double, _dp, _dp, _dp]
    L.orc_ck_attempt.argtypes = [i3, d3, i3, C.c_double, _dp, _dp, C.c_double, _dp, d3, C.c_void_p]
    L.orc_convexity.argtypes = [i3, d3, i3, _dp, C.c_void_p, C.POINTER(C.c_long)]
    L.orc_convexity.restype = C.c_int
    L.orc_controller.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, d3]
    L.orc_run.argtypes = [i3, d3, i3, C.c_double, C.c_double, C.c_int, C.c_double, C.c_double, C.c_double,
                          C.c_int, _dp, _dp, d3, d3, C.c_void_p, C.c_void_p, C.POINTER(C.c_int)]
    L.orcz_run_fixed.argtypes = [i3, d3, i3, C.c_double, C.c_int, _dp, _zp, _zp, C.c_void_p, C.c_void_p]
    L.orc_rhs_sampled.argtypes = [i3, d3, i3, C.c_double, _dp, _dp, C.c_long,
                                  np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS"), _dp]
    L.orc_rhs_sampled.restype = C.c_int
    L.orc_set_curl.argtypes = [C.c_int]
    L.orc_set_curl.restype = C.c_int
    L.orc_threads.argtypes = []
    L.orc_threads.restype = C.c_int
    L.orc_set_threads.argtypes = [C.c_int]
    L.orc_set_threads.restype = None
    L.orc_tableau.argtypes = [_dp, _dp, _dp]
    L.orc_tableau.restype = None
    for f in (L.orc_fields, L.orc_diagnostics, L.orc_ck_attempt, L.orc_controller, L.orc_run, L.orcz_run_fixed):
        f.restype = C.c_int
    _lib = L
    return L


def _g(grid):
    n = (C.c_int * 3)(*[int(v) for v in grid.n])
    h = (C.c_double * 3)(*[float(v) for v in grid.h])
    bc = (C.c_int * 3)(*[int(v) for v in grid.bc])
    return n, h, bc


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _vec(grid, a, name="field"):
    """a as a contiguous FP64 [3][nz][ny][nx] array of this grid (shape checked)."""
    a = _f64(a)
    want = (3, int(grid.n[2]), int(grid.n[1]), int(grid.n[0]))
    if a.shape != want:
        raise ValueError(f"{name} has shape {a.shape}, expected {want}")
    return a


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__(f"oracle status {code}")
        self.code = code


def _check(rc):
    if rc != OK:
        raise OracleError(rc)


def fields(grid, x, B0, gamma=1.0):
    """B, Delta, J, u at every node of positions x (J and u are zero on line-tied faces)."""
    x, B0 = _vec(grid, x, "x"), _vec(grid, B0, "B0")
    shp = x.shape
    B, J, u = np.empty(shp), np.empty(shp), np.empty(shp)
    det = np.empty(shp[1:])
    _check(lib().orc_fields(*_g(grid), gamma, x, B0, _ptr(B), _ptr(det), _ptr(J), _ptr(u)))
    return {"B": B, "det": det, "J": J, "u": u}


def alpha_star(grid, x, B0):
    """alpha* = J.B / |B|^2 at every node (Sec. 3.2.1), with B and J of fields(); 0 where B = 0
    (and on line-tied faces, where J is zero).  Shape (nz, ny, nx)."""
    f = fields(grid, x, B0)
    B, J = f["B"], f["J"]
    B2 = B[0] * B[0] + B[1] * B[1] + B[2] * B[2]
    JB = J[0] * B[0] + J[1] * B[1] + J[2] * B[2]
    out = np.zeros_like(B2)
    np.divide(JB, B2, out=out, where=B2 > 0)
    return out


def convexity(grid, x):
    """(kappa (nz, ny, nx) int array of +1 / -1, number of concave nodes) of positions x."""
    x = _vec(grid, x, "x")
    kappa = np.empty(x.shape[1:], dtype=np.int32)
    count = C.c_long(0)
    _check(lib().orc_convexity(*_g(grid), x, kappa.ctypes.data_as(C.c_void_p), C.byref(count)))
    return kappa, int(count.value)


def rhs_sampled(grid, x, B0, nodes, gamma=1.0):
    """u at the given flat node indices (k*ny + j)*nx + i; returns (len(nodes), 3)."""
    nodes = np.ascontiguousarray(nodes, dtype=np.int64)
    out = np.zeros((len(nodes), 3))
    _check(lib().orc_rhs_sampled(*_g(grid), gamma, _f64(x), _f64(B0), len(nodes), nodes, out))
    return out


def diagnostics(grid, x, B0, tau_B2=0.0):
    """{E_M, xi, min_det, R2, skipped} of positions x."""
    out = np.zeros(5)
    _check(lib().orc_diagnostics(*_g(grid), float(tau_B2), _vec(grid, x, "x"), _vec(grid, B0, "B0"), out))
    return {"E_M": out[0], "xi": out[1], "min_det": out[2], "R2": out[3], "skipped": int(out[4])}


def ck_attempt(grid, x, B0, dt, gamma=1.0, want_k=False):
    """One Cash-Karp attempt with fixed dt: (x_new, Lambda[, k (6,3,nz,ny,nx)])."""
    x, B0 = _f64(x), _f64(B0)
    xn = np.empty_like(x)
    lam = C.c_double(0.0)
    k = np.empty((6,) + x.shape) if want_k else None
    _check(lib().orc_ck_attempt(*_g(grid), gamma, x, B0, float(dt), xn, C.byref(lam), _ptr(k)))
    return (xn, lam.value, k) if want_k else (xn, lam.value)


CURL_NN, CURL_NNN = 0, 1


@contextlib.contextmanager
def curl(kind: int):
    """Inside the block every call computes the current with the given operator: CURL_NN, the
    nearest-neighbour loops of Sec. 2.2 (the default), or CURL_NNN, the next-nearest-neighbour
    octilateral of Sec. 2.3."""
    _check(lib().orc_set_curl(int(kind)))
    try:
        yield
    finally:
        lib().orc_set_curl(CURL_NN)


def threads() -> int:
    """OpenMP threads the oracle's sweeps use."""
    return int(lib().orc_threads())


def set_threads(n: int) -> None:
    """OpenMP threads of the oracle's later sweeps (for timing it on a given core count)."""
    lib().orc_set_threads(int(n))


def tableau():
    """(A (6x6), b5 (6), b4 (6)) exactly as the oracle stores them."""
    A, b5, b4 = np.zeros(36), np.zeros(6), np.zeros(6)
    lib().orc_tableau(A, b5, b4)
    return A.reshape(6, 6), b5, b4


def controller(dt, Lambda, tol, safety=1.0):
    """Step-size rule: (accepted, dt_next)."""
    out = C.c_double(0.0)
    acc = lib().orc_controller(float(dt), float(Lambda), float(tol), float(safety), C.byref(out))
    return bool(acc), out.value


MODE_FIXED, MODE_ADAPTIVE, MODE_REPLAY = 0, 1, 2


def run(grid, x0, B0, K, dt, mode=MODE_ADAPTIVE, tol=1e-7, dt_min=1e-12, t=0.0, tau_B2=0.0, gamma=1.0,
        dts=None, raise_on_error=True, safety=1.0):
    """K accepted steps from x0.  Returns dict(x, t, dt, diag (K,8), status, done).

    diag columns: t, dt used, E_M, xi, R2, Lambda, min Delta, rejects (pre-step state).
    """
    x = _vec(grid, x0, "x0").copy()
    B0 = _vec(grid, B0, "B0")
    tt, dd = C.c_double(t), C.c_double(dt)
    diag = np.zeros((max(K, 1), 8))
    done = C.c_int(0)
    dts_arr = None if dts is None else _f64(dts)
    rc = lib().orc_run(*_g(grid), gamma, float(tau_B2), int(mode), float(tol), float(safety), float(dt_min), int(K),
                       x, B0,
                       C.byref(tt), C.byref(dd), _ptr(dts_arr), _ptr(diag), C.byref(done))
    if raise_on_error and rc != OK:
        raise OracleError(rc)
    return {"x": x, "t": tt.value, "dt": dd.value, "diag": diag[:done.value], "status": rc, "done": done.value}


def run_fixed_complex(grid, x0, B0, dts, gamma=1.0):
    """Fixed-dt trajectory in complex arithmetic: (E_M, R2) of the final state, complex."""
    x = np.ascontiguousarray(x0, dtype=np.complex128).copy()
    B0 = np.ascontiguousarray(B0, dtype=np.complex128)
    dts = _f64(dts)
    E = np.zeros(1, dtype=np.complex128)
    R = np.zeros(1, dtype=np.complex128)
    _check(lib().orcz_run_fixed(*_g(grid), gamma, len(dts), dts, x, B0, _ptr(E), _ptr(R)))
    return complex(E[0]), complex(R[0])


def null_threshold(B0, tau=1e-12):
    """Absolute |B|^2 threshold of the xi null guard: tau * max_nodes |B0|^2."""
    B0 = np.asarray(B0)
    return float(tau * (B0 ** 2).sum(axis=0).max())
