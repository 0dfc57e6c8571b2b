"""ctypes wrapper of the FP64 CPU oracle (spoly_oracle.c, tail_oracle.c).

TEST INFRASTRUCTURE: only the test-suite, the smoke check and the CPU-baseline
leg of the benchmark import this module.  It takes plain numpy arrays; it does
not import the HIP package.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRCS = [os.path.join(HERE, "spoly_oracle.c"), os.path.join(HERE, "tail_oracle.c")]
LIB = os.path.join(HERE, "liboracle.so")

SOL_DTYPE = np.dtype([("query", np.int32), ("flags", np.int32), ("u1", np.float64), ("v1", np.float64),
                      ("u2", np.float64), ("v2", np.float64), ("residual", np.float64), ("edge", np.float64)])
DIAG_DTYPE = np.dtype([("n_vroots", np.int32), ("n_cand", np.int32), ("n_valid", np.int32), ("flags", np.int32),
                       ("tangency", np.float64), ("min_gap", np.float64)])

F_DEGENERATE, F_EDGE2, F_AXIS_Z, F_AXIS_Y, F_FLAT1, F_FLAT2 = 1, 2, 4, 8, 16, 32


class Params(ctypes.Structure):
    _fields_ = [("tau", ctypes.c_double), ("u_margin", ctypes.c_double), ("dedup", ctypes.c_double),
                ("polish_iters", ctypes.c_int32), ("pieces", ctypes.c_int32),
                ("bisect_iters", ctypes.c_int32), ("det_method", ctypes.c_int32)]


class SqrtFit(ctypes.Structure):
    _fields_ = [("bp", ctypes.c_double * 7), ("c", (ctypes.c_double * 4) * 6)]


def default_params(two_bounce: bool = False) -> Params:
    """Readings of the constants: tau = 1e-6 on |h^ x n^|; 100 pieces and 10
    bisection steps (Sec. 5.2); u searched on [-m, 1-v+m] before polish with
    m = 1e-4 (one bounce) or 0.05 (two bounces, whose approximate roots can sit
    up to ~1e-2 away from the exact ones); up to 6 Newton steps; two vertices
    take the sign of det R(v) from the paired product formula with b evaluated
    from its defining products and the roots at x2 = infinity left out
    (det_method 3; 2 is the same on expanded coefficients, 1 the plain
    product, 0 Gaussian elimination on the Bezout matrix)."""
    return Params(1e-6, 0.05 if two_bounce else 1e-4, 1e-8, 6, 100, 10, 3 if two_bounce else 0)


def build(force: bool = False) -> str:
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < max(os.path.getmtime(s) for s in SRCS):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-o", tmp, *SRCS, "-lm"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(LIB)
        P = ctypes.c_void_p
        L.or_solve_1bounce.argtypes = [P, P, P, ctypes.c_int64, P, P, P, P, P, ctypes.c_int64, ctypes.c_int32,
                                       ctypes.c_double, ctypes.c_double, P, P, P, P]
        L.or_solve_tt.argtypes = [P, P, P, ctypes.c_int64, P, P, P, P, P, P, ctypes.c_int64, P, P, P, P, P, P]
        L.or_solve_2v.argtypes = [P, P, P, ctypes.c_int64, P, P, P, P, P, P, ctypes.c_int64, P, P, P, P, P, P, P]
        L.or_coeffs_2v.argtypes = [P, P, P, ctypes.c_int64, ctypes.c_int64, P, P, P, P, P, P, P, P, P, P, P]
        L.or_coeffs_1bounce.argtypes = [P, P, P, ctypes.c_int64, P, P, ctypes.c_int32, ctypes.c_double,
                                        ctypes.c_double, P, P, P, P, P, P]
        L.or_coeffs_tt.argtypes = [P, P, P, ctypes.c_int64, ctypes.c_int64, P, P, P, P, P, P, P, P, P, P]
        L.or_resultant_laplace.argtypes = [P, ctypes.c_int32, P, ctypes.c_int32, ctypes.c_int32, P]
        L.or_isolate.argtypes = [P, ctypes.c_int32, ctypes.c_double, ctypes.c_double, P, ctypes.c_int32]
        L.or_det_sign.argtypes = [P, ctypes.c_int32, P, ctypes.c_int32, ctypes.c_int32, ctypes.c_double]
        L.or_res_sign.argtypes = [P, ctypes.c_int32, P, ctypes.c_int32, ctypes.c_int32, ctypes.c_double]
        L.or_res_sign_paired.argtypes = [P, ctypes.c_int32, P, ctypes.c_int32, ctypes.c_int32, ctypes.c_double]
        L.or_maxsol.restype = ctypes.c_int
        L.or_set_threads.argtypes = [ctypes.c_int]
        L.or_set_threads.restype = ctypes.c_int
        L.or_opcount_1bounce.argtypes = [P, P, P, P, P, P, P, P, ctypes.c_int64, ctypes.c_int32, ctypes.c_double,
                                         ctypes.c_double, P, P]
        L.or_opcount_2v.argtypes = [P, P, P, P, P, P, P, P, P, ctypes.c_int64, P, P, P, P, P]
        L.or_cull_tt.argtypes = [P, P, P, ctypes.c_int64, P, ctypes.c_int64, P, ctypes.c_int64, P,
                                 ctypes.c_double, P]
        L.or_cull_1bounce.argtypes = [P, P, P, ctypes.c_int64, P, ctypes.c_int64, P, ctypes.c_int64,
                                      ctypes.c_double, ctypes.c_double, ctypes.c_double, P]
        L.ot_tail.argtypes = [P, P, P, ctypes.c_int64, P, P, P, P, P, P, P, ctypes.c_int64, ctypes.c_int32, P, P,
                              ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double, P, P, P, P, P]
        L.ot_seg_tri.argtypes = [P, P, P, P, P, ctypes.c_int64, ctypes.c_double, P, P]
        L.ot_fresnel_t.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double]
        L.ot_fresnel_t.restype = ctypes.c_double
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def set_threads(n: int) -> int:
    """Host threads of the parallel solves; returns the previous count."""
    return int(lib().or_set_threads(int(n)))


def maxsol() -> int:
    return lib().or_maxsol()


def solve_1bounce(P, N, tri, x0s, x2s, q_x0, q_x2, q_tri, event: str, eta0: float = 1.0, eta1: float = 1.0,
                  params: Params | None = None):
    """Returns (solutions structured array sorted by (query, v1, u1), diag per query)."""
    L = lib()
    P, N, x0s, x2s = (_c(a, np.float64) for a in (P, N, x0s, x2s))
    tri, q_x0, q_x2, q_tri = (_c(a, np.int32) for a in (tri, q_x0, q_x2, q_tri))
    nq = len(q_tri)
    ms = maxsol()
    out = np.zeros(nq * ms, dtype=SOL_DTYPE)
    cnt = np.zeros(nq, dtype=np.int32)
    diag = np.zeros(nq, dtype=DIAG_DTYPE)
    prm = params or default_params(False)
    L.or_solve_1bounce(_p(P), _p(N), _p(tri), len(tri), _p(x0s), _p(x2s), _p(q_x0), _p(q_x2), _p(q_tri), nq,
                       1 if event == "T" else 0, eta0, eta1, ctypes.byref(prm), _p(out), _p(cnt), _p(diag))
    sel = (np.arange(ms)[None, :] < cnt[:, None]).ravel()
    sols = out[sel]
    sols = sols[np.lexsort((sols["u1"], sols["v1"], sols["query"]))]
    return sols, diag


def sqrt_fit_struct(coefs=None, breakpoints=None) -> SqrtFit:
    from sqrt_fit import BREAKPOINTS, fit_table  # noqa: local module of the oracle

    if coefs is None:
        coefs, _ = fit_table()
    bp = breakpoints or BREAKPOINTS
    s = SqrtFit()
    for i in range(7):
        s.bp[i] = bp[i]
    for i in range(6):
        for j in range(4):
            s.c[i][j] = float(coefs[i][j])
    return s


_fit_cache = None


def default_sqrt_fit() -> SqrtFit:
    global _fit_cache
    if _fit_cache is None:
        _fit_cache = sqrt_fit_struct()
    return _fit_cache


def _chain(chain: str) -> np.ndarray:
    assert len(chain) == 2 and set(chain) <= {"R", "T"}, chain
    return np.array([0 if c == "R" else 1 for c in chain], dtype=np.int32)


def solve_2v(P, N, tri, x0s, x3s, q_x0, q_x3, q_t1, q_t2, chain: str, eta=(1.0, 1.5, 1.0),
             params: Params | None = None, fit: SqrtFit | None = None):
    """Two specular vertices; chain "RR", "RT", "TR" or "TT" (event at x1, then at x2)."""
    L = lib()
    P, N, x0s, x3s = (_c(a, np.float64) for a in (P, N, x0s, x3s))
    tri, q_x0, q_x3, q_t1, q_t2 = (_c(a, np.int32) for a in (tri, q_x0, q_x3, q_t1, q_t2))
    nq = len(q_t1)
    ms = maxsol()
    out = np.zeros(nq * ms, dtype=SOL_DTYPE)
    cnt = np.zeros(nq, dtype=np.int32)
    diag = np.zeros(nq, dtype=DIAG_DTYPE)
    eta = _c(eta, np.float64)
    ch = _chain(chain)
    prm = params or default_params(True)
    fit = fit or default_sqrt_fit()
    L.or_solve_2v(_p(P), _p(N), _p(tri), len(tri), _p(x0s), _p(x3s), _p(q_x0), _p(q_x3), _p(q_t1), _p(q_t2), nq,
                  _p(eta), _p(ch), ctypes.byref(fit), ctypes.byref(prm), _p(out), _p(cnt), _p(diag))
    sel = (np.arange(ms)[None, :] < cnt[:, None]).ravel()
    sols = out[sel]
    sols = sols[np.lexsort((sols["u1"], sols["v1"], sols["query"]))]
    return sols, diag


def coeffs_2v(P, N, tri, t1: int, t2: int, x0, x3, chain: str, eta=(1.0, 1.5, 1.0), fit: SqrtFit | None = None):
    L = lib()
    P, N = _c(P, np.float64), _c(N, np.float64)
    tri = _c(tri, np.int32)
    x0 = _c(x0, np.float64).reshape(3)
    x3 = _c(x3, np.float64).reshape(3)
    eta = _c(eta, np.float64)
    ch = _chain(chain)
    fit = fit or default_sqrt_fit()
    a = np.zeros(49 * 49)
    b = np.zeros(49 * 49)
    da, db, nb, fl = (ctypes.c_int32() for _ in range(4))
    L.or_coeffs_2v(_p(P), _p(N), _p(tri), int(t1), int(t2), _p(x0), _p(x3), _p(eta), _p(ch), ctypes.byref(fit),
                   _p(a), ctypes.byref(da), _p(b), ctypes.byref(db), ctypes.byref(nb), ctypes.byref(fl))
    A = a[:(da.value + 1) ** 2].reshape(da.value + 1, da.value + 1)
    B = b[:(db.value + 1) ** 2].reshape(db.value + 1, db.value + 1)
    return A, B, nb.value, fl.value


def solve_tt(P, N, tri, x0s, x3s, q_x0, q_x3, q_t1, q_t2, eta=(1.0, 1.5, 1.0), params: Params | None = None,
             fit: SqrtFit | None = None):
    L = lib()
    P, N, x0s, x3s = (_c(a, np.float64) for a in (P, N, x0s, x3s))
    tri, q_x0, q_x3, q_t1, q_t2 = (_c(a, np.int32) for a in (tri, q_x0, q_x3, q_t1, q_t2))
    nq = len(q_t1)
    ms = maxsol()
    out = np.zeros(nq * ms, dtype=SOL_DTYPE)
    cnt = np.zeros(nq, dtype=np.int32)
    diag = np.zeros(nq, dtype=DIAG_DTYPE)
    eta = _c(eta, np.float64)
    prm = params or default_params(True)
    fit = fit or default_sqrt_fit()
    L.or_solve_tt(_p(P), _p(N), _p(tri), len(tri), _p(x0s), _p(x3s), _p(q_x0), _p(q_x3), _p(q_t1), _p(q_t2), nq,
                  _p(eta), ctypes.byref(fit), ctypes.byref(prm), _p(out), _p(cnt), _p(diag))
    sel = (np.arange(ms)[None, :] < cnt[:, None]).ravel()
    sols = out[sel]
    sols = sols[np.lexsort((sols["u1"], sols["v1"], sols["query"]))]
    return sols, diag


def opcount_1bounce(P, N, tri, x0s, x2s, q_x0, q_x2, q_tri, event: str, eta0=1.0, eta1=1.0,
                    params: Params | None = None) -> np.ndarray:
    """Op counts [nq, 4] by stage (coefficients, elimination, root finding in v,
    path phase) of each one-vertex query."""
    L = lib()
    P, N, x0s, x2s = (_c(a, np.float64) for a in (P, N, x0s, x2s))
    tri, q_x0, q_x2, q_tri = (_c(a, np.int32) for a in (tri, q_x0, q_x2, q_tri))
    nq = len(q_tri)
    ops = np.zeros(4 * nq, dtype=np.uint64)
    prm = params or default_params(False)
    L.or_opcount_1bounce(_p(P), _p(N), _p(tri), _p(x0s), _p(x2s), _p(q_x0), _p(q_x2), _p(q_tri), nq,
                         1 if event == "T" else 0, eta0, eta1, ctypes.byref(prm), _p(ops))
    return ops.reshape(nq, 4)


def opcount_2v(P, N, tri, x0s, x3s, q_x0, q_x3, q_t1, q_t2, chain: str, eta=(1.0, 1.5, 1.0),
               params: Params | None = None, fit: SqrtFit | None = None) -> np.ndarray:
    """Op counts [nq, 4] by stage (coefficients, scan samples, bisection
    samples, path phase) of each two-vertex query."""
    L = lib()
    P, N, x0s, x3s = (_c(a, np.float64) for a in (P, N, x0s, x3s))
    tri, q_x0, q_x3, q_t1, q_t2 = (_c(a, np.int32) for a in (tri, q_x0, q_x3, q_t1, q_t2))
    nq = len(q_t1)
    ops = np.zeros(4 * nq, dtype=np.uint64)
    eta = _c(eta, np.float64)
    ch = _chain(chain)
    prm = params or default_params(True)
    fit = fit or default_sqrt_fit()
    L.or_opcount_2v(_p(P), _p(N), _p(tri), _p(x0s), _p(x3s), _p(q_x0), _p(q_x3), _p(q_t1), _p(q_t2), nq,
                    _p(eta), _p(ch), ctypes.byref(fit), ctypes.byref(prm), _p(ops))
    return ops.reshape(nq, 4)


def coeffs_1bounce(P, N, tri, t: int, x0, x2, event: str, eta0=1.0, eta1=1.0):
    """Dense bivariate coefficient arrays A[i,j] (u^i v^j) of a and b, the Bezout size and flags."""
    L = lib()
    P, N = _c(P, np.float64), _c(N, np.float64)
    tri = _c(tri, np.int32)
    x0 = _c(x0, np.float64).reshape(3)
    x2 = _c(x2, np.float64).reshape(3)
    a = np.zeros(49 * 49)
    b = np.zeros(49 * 49)
    da, db, nb, fl = (ctypes.c_int32() for _ in range(4))
    L.or_coeffs_1bounce(_p(P), _p(N), _p(tri), int(t), _p(x0), _p(x2), 1 if event == "T" else 0, eta0, eta1,
                        _p(a), ctypes.byref(da), _p(b), ctypes.byref(db), ctypes.byref(nb), ctypes.byref(fl))
    A = a[:(da.value + 1) ** 2].reshape(da.value + 1, da.value + 1)
    B = b[:(db.value + 1) ** 2].reshape(db.value + 1, db.value + 1)
    return A, B, nb.value, fl.value


def coeffs_tt(P, N, tri, t1: int, t2: int, x0, x3, eta=(1.0, 1.5, 1.0), fit: SqrtFit | None = None):
    L = lib()
    P, N = _c(P, np.float64), _c(N, np.float64)
    tri = _c(tri, np.int32)
    x0 = _c(x0, np.float64).reshape(3)
    x3 = _c(x3, np.float64).reshape(3)
    eta = _c(eta, np.float64)
    fit = fit or default_sqrt_fit()
    a = np.zeros(49 * 49)
    b = np.zeros(49 * 49)
    da, db, nb, fl = (ctypes.c_int32() for _ in range(4))
    L.or_coeffs_tt(_p(P), _p(N), _p(tri), int(t1), int(t2), _p(x0), _p(x3), _p(eta), ctypes.byref(fit),
                   _p(a), ctypes.byref(da), _p(b), ctypes.byref(db), ctypes.byref(nb), ctypes.byref(fl))
    A = a[:(da.value + 1) ** 2].reshape(da.value + 1, da.value + 1)
    B = b[:(db.value + 1) ** 2].reshape(db.value + 1, db.value + 1)
    return A, B, nb.value, fl.value


def resultant_laplace(A: np.ndarray, B: np.ndarray, n: int) -> np.ndarray:
    L = lib()
    A = _c(A, np.float64)
    B = _c(B, np.float64)
    r = np.zeros(256)
    d = L.or_resultant_laplace(_p(A), A.shape[0] - 1, _p(B), B.shape[0] - 1, n, _p(r))
    return r[:d + 1] if d >= 0 else np.zeros(0)


def isolate(c, lo: float, hi: float) -> np.ndarray:
    L = lib()
    c = _c(c, np.float64)
    out = np.zeros(max(len(c), 1) + 4)
    n = L.or_isolate(_p(c), len(c) - 1, lo, hi, _p(out), len(out))
    return out[:n].copy()


def det_sign(A: np.ndarray, B: np.ndarray, n: int, v: float) -> int:
    L = lib()
    A = _c(A, np.float64)
    B = _c(B, np.float64)
    return int(L.or_det_sign(_p(A), A.shape[0] - 1, _p(B), B.shape[0] - 1, n, v))


def res_sign(A: np.ndarray, B: np.ndarray, ma: int, v: float) -> int:
    """Sign of det R(v) by the product formula (det_method 1): product of
    sgn b(alpha, v) over all real roots alpha of a(., v), whose u-degree is ma."""
    L = lib()
    A = _c(A, np.float64)
    B = _c(B, np.float64)
    return int(L.or_res_sign(_p(A), A.shape[0] - 1, _p(B), B.shape[0] - 1, int(ma), v))


def res_sign_paired(A: np.ndarray, B: np.ndarray, ma: int, v: float) -> int:
    """The two-vertex default (det_method 2): the product of sgn b(alpha, v)
    over the real roots alpha of a(., v), two consecutive roots closer than
    1e-4 max(1, |alpha|) left out."""
    L = lib()
    A = _c(A, np.float64)
    B = _c(B, np.float64)
    return int(L.or_res_sign_paired(_p(A), A.shape[0] - 1, _p(B), B.shape[0] - 1, int(ma), v))


def cull_1bounce(P, N, tri, x0s, x2s, eta0=1.0, eta1=1.0, margin=0.0) -> np.ndarray:
    """Keep mask [n0, n2, nt] (bool) of the FP64 normal-cone cull."""
    L = lib()
    P, N, x0s, x2s = (_c(a, np.float64) for a in (P, N, x0s, x2s))
    tri = _c(tri, np.int32)
    n0, n2, nt = len(x0s), len(x2s), len(tri)
    keep = np.zeros(n0 * n2 * nt, dtype=np.uint8)
    L.or_cull_1bounce(_p(P), _p(N), _p(tri), nt, _p(x0s), n0, _p(x2s), n2, eta0, eta1, margin, _p(keep))
    return keep.reshape(n0, n2, nt).astype(bool)


def cull_tt(P, N, tri, x0s, x3s, eta=(1.0, 1.5, 1.0), margin=0.0) -> np.ndarray:
    """Keep mask [n0, n3, nt, nt] (bool) of the FP64 two-vertex cone cull."""
    L = lib()
    P, N, x0s, x3s = (_c(a, np.float64) for a in (P, N, x0s, x3s))
    tri = _c(tri, np.int32)
    eta = _c(eta, np.float64)
    n0, n3, nt = len(x0s), len(x3s), len(tri)
    keep = np.zeros(n0 * n3 * nt * nt, dtype=np.uint8)
    L.or_cull_tt(_p(P), _p(N), _p(tri), nt, _p(x0s), n0, _p(x3s), n3, _p(eta), margin, _p(keep))
    return keep.reshape(n0, n3, nt, nt).astype(bool)


# ------------------------------------------------------------------ path-phase tail (tail_oracle.c)

TAIL_DTYPE = np.dtype([("mask", np.int32), ("margin", np.float64), ("fresnel", np.float64), ("E", np.float64),
                       ("E_change", np.float64)])


def tail(P, N, tri, x0s, xls, q_x0, q_xl, ptri, pu, pv, chain: str, eta, intensity=1.0, rho=1.0, teps=1e-6,
         h=1e-6) -> np.ndarray:
    """Visibility and contribution of n paths with k = len(chain) vertices.
    ptri, pu, pv: [n, k] triangle ids and barycentrics of x1..xk; q_x0, q_xl:
    receiver and light index per path; eta: k+1 indices (eta[i] between x_i
    and x_{i+1}).  Returns a TAIL_DTYPE record per path."""
    L = lib()
    k = len(chain)
    assert k in (1, 2) and set(chain) <= {"R", "T"} and len(eta) == k + 1
    P, N, x0s, xls = (_c(a, np.float64) for a in (P, N, x0s, xls))
    tri, q_x0, q_xl = (_c(a, np.int32) for a in (tri, q_x0, q_xl))
    ptri = _c(np.asarray(ptri).reshape(-1, k), np.int32)
    pu = _c(np.asarray(pu).reshape(-1, k), np.float64)
    pv = _c(np.asarray(pv).reshape(-1, k), np.float64)
    n = len(ptri)
    ev = np.array([0 if c == "R" else 1 for c in chain], dtype=np.int32)
    eta = _c(eta, np.float64)
    out = {f: np.zeros(n, dtype=TAIL_DTYPE[f]) for f in TAIL_DTYPE.names}
    L.ot_tail(_p(P), _p(N), _p(tri), len(tri), _p(x0s), _p(xls), _p(q_x0), _p(q_xl), _p(ptri), _p(pu), _p(pv), n,
              k, _p(ev), _p(eta), float(intensity), float(rho), float(teps), float(h),
              *(_p(out[f]) for f in TAIL_DTYPE.names))
    rec = np.zeros(n, dtype=TAIL_DTYPE)
    for f in TAIL_DTYPE.names:
        rec[f] = out[f]
    return rec


def seg_tri(p, q, a, b, c, teps=0.0):
    """Moller-Trumbore segment/triangle test per row; returns (hit, margin)."""
    L = lib()
    p, q, a, b, c = (_c(np.asarray(x).reshape(-1, 3), np.float64) for x in (p, q, a, b, c))
    n = len(p)
    hit = np.zeros(n, dtype=np.int32)
    margin = np.zeros(n)
    L.ot_seg_tri(_p(p), _p(q), _p(a), _p(b), _p(c), n, float(teps), _p(hit), _p(margin))
    return hit.astype(bool), margin


def fresnel_t(n1: float, n2: float, ci: float) -> float:
    return float(lib().ot_fresnel_t(float(n1), float(n2), float(ci)))
