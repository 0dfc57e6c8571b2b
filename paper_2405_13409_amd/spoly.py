"""Python binding of libspoly.so (include/spoly.h): argument marshalling only.

Device memory and streams come from PyTorch; every step of the solve runs in
the library's HIP kernels.  The library must be built (``build.py``); loading
fails loudly otherwise.  torch is imported before the library is opened so
that both share torch's HIP runtime.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libspoly.so")

SPOLY_OK, SPOLY_E_INVALID_ARG, SPOLY_E_CAPACITY, SPOLY_E_DEVICE, SPOLY_E_UNSUPPORTED = range(5)
SPOLY_R, SPOLY_T = 0, 1
SPOLY_FP64, SPOLY_FP32_POLISH64 = 0, 1

SOLUTION_DTYPE = np.dtype([("query", "<i4"), ("tri", "<i4", (2,)), ("flags", "<u4"), ("u", "<f8", (2,)),
                           ("v", "<f8", (2,)), ("residual", "<f4"), ("edge", "<f4")])
assert SOLUTION_DTYPE.itemsize == 56

EXPORTED = ("spoly_ctx_create", "spoly_ctx_destroy", "spoly_default_params", "spoly_status_str",
            "spoly_cull_1bounce", "spoly_solve_1bounce", "spoly_cull_2bounce", "spoly_solve_nbounce",
            "spoly_prune_score", "spoly_pruner_fwd_bwd", "spoly_pruner_step", "spoly_pruner_features",
            "spoly_solve_mixed", "spoly_tt_default_params", "spoly_solve_1bounce_noalloc", "spoly_stage_times",
            "spoly_bvh_build", "spoly_bvh_destroy", "spoly_tail_default_params", "spoly_path_tail")
SPOLY_FLAG_FORCE_FP64 = 1 << 1
SPOLY_FLAG_STAGE_TIMES = 1 << 2
SPOLY_FLAG_DETERMINISTIC_ORDER = 1 << 3
PRUNER_NPARAMS = 38657


class SpolyError(RuntimeError):
    pass


class Mesh(ctypes.Structure):
    _fields_ = [("px", ctypes.c_void_p), ("py", ctypes.c_void_p), ("pz", ctypes.c_void_p),
                ("nx", ctypes.c_void_p), ("ny", ctypes.c_void_p), ("nz", ctypes.c_void_p),
                ("tri", ctypes.c_void_p), ("n_vertices", ctypes.c_int32), ("n_tris", ctypes.c_int32)]


class Points(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p), ("y", ctypes.c_void_p), ("z", ctypes.c_void_p), ("n", ctypes.c_int32)]


class MixedShape(ctypes.Structure):
    _fields_ = [("workgroups_per_cu", ctypes.c_int32), ("r_tile", ctypes.c_int32), ("order", ctypes.c_int32),
                ("pad", ctypes.c_int32)]


class Params(ctypes.Structure):
    _fields_ = [("pieces", ctypes.c_int32), ("bisect_iters", ctypes.c_int32), ("iso_eps", ctypes.c_double),
                ("tau", ctypes.c_double), ("u_margin", ctypes.c_double), ("dedup", ctypes.c_double),
                ("polish_iters", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class TailParams(ctypes.Structure):
    _fields_ = [("intensity", ctypes.c_double), ("reflectance", ctypes.c_double), ("t_eps", ctypes.c_double),
                ("rcv_normal", ctypes.c_double * 3)]


TAIL_SINGULAR = 1 << 30

_lib = None


def load_library(path: str = LIB_PATH):
    """Open libspoly.so (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise SpolyError(f"{path} is missing: build it with `python -m paper_2405_13409_amd.build`")
    L = ctypes.CDLL(path)
    P, I32, I64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    L.spoly_ctx_create.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int]
    L.spoly_ctx_create.restype = ctypes.c_int
    L.spoly_ctx_destroy.argtypes = [P]
    L.spoly_ctx_destroy.restype = None
    L.spoly_default_params.argtypes = [ctypes.POINTER(Params)]
    L.spoly_default_params.restype = None
    L.spoly_tt_default_params.argtypes = [ctypes.POINTER(Params)]
    L.spoly_tt_default_params.restype = None
    L.spoly_status_str.argtypes = [ctypes.c_int]
    L.spoly_status_str.restype = ctypes.c_char_p
    L.spoly_stage_times.argtypes = [P, P, ctypes.c_int32]
    L.spoly_stage_times.restype = ctypes.c_int32
    L.spoly_cull_1bounce.argtypes = [P, ctypes.POINTER(Mesh), ctypes.POINTER(Points), ctypes.POINTER(Points), D, D, D,
                                     P, P, P, I64, P, P]
    L.spoly_cull_1bounce.restype = ctypes.c_int
    L.spoly_solve_1bounce.argtypes = [P, ctypes.POINTER(Mesh), ctypes.POINTER(Points), ctypes.POINTER(Points), P, P, P,
                                      I64, ctypes.c_int, D, D, ctypes.c_int, ctypes.POINTER(Params), P, I64, P, P, P, P]
    L.spoly_solve_1bounce.restype = ctypes.c_int
    L.spoly_solve_1bounce_noalloc.argtypes = [ctypes.POINTER(Mesh), ctypes.POINTER(Points), ctypes.POINTER(Points),
                                              P, P, P, I64, ctypes.c_int, D, D, ctypes.c_int, ctypes.POINTER(Params),
                                              P, I64, P, P, P, P]
    L.spoly_solve_1bounce_noalloc.restype = ctypes.c_int
    L.spoly_cull_2bounce.argtypes = [P, ctypes.POINTER(Mesh), ctypes.POINTER(Points), ctypes.POINTER(Points), P, D,
                                     P, P, P, P, I64, P, P]
    L.spoly_cull_2bounce.restype = ctypes.c_int
    L.spoly_solve_nbounce.argtypes = [P, ctypes.POINTER(Mesh), I32, P, P, ctypes.POINTER(Points),
                                      ctypes.POINTER(Points), P, P, P, I64, ctypes.c_int, ctypes.POINTER(Params), P, P,
                                      I64, P, P, P, P]
    L.spoly_solve_nbounce.restype = ctypes.c_int
    F = ctypes.c_float
    MP, PP = ctypes.POINTER(Mesh), ctypes.POINTER(Points)
    L.spoly_prune_score.argtypes = [P, MP, PP, PP, P, P, P, I64, P, F, P, P, I64, P, P]
    L.spoly_prune_score.restype = ctypes.c_int
    L.spoly_pruner_fwd_bwd.argtypes = [P, MP, PP, PP, P, P, P, I64, P, F, P, P, P, P]
    L.spoly_pruner_fwd_bwd.restype = ctypes.c_int
    L.spoly_pruner_step.argtypes = [P, P, P, P, P, I64, F, F, F, F, P]
    L.spoly_pruner_step.restype = ctypes.c_int
    L.spoly_pruner_features.argtypes = [P, MP, PP, PP, P, P, P, I64, P, P]
    L.spoly_pruner_features.restype = ctypes.c_int
    L.spoly_solve_mixed.argtypes = [P, MP, PP, PP, P, P, P, I64, ctypes.c_int, D, D, MP, PP, PP, P, P, P, I64, P,
                                    ctypes.c_int, ctypes.POINTER(Params), ctypes.POINTER(MixedShape), P, P, I64, P, P]
    L.spoly_solve_mixed.restype = ctypes.c_int
    L.spoly_bvh_build.argtypes = [P, MP, ctypes.POINTER(ctypes.c_void_p), P]
    L.spoly_bvh_build.restype = ctypes.c_int
    L.spoly_bvh_destroy.argtypes = [P]
    L.spoly_bvh_destroy.restype = None
    L.spoly_tail_default_params.argtypes = [ctypes.POINTER(TailParams)]
    L.spoly_tail_default_params.restype = None
    L.spoly_path_tail.argtypes = [P, MP, P, I32, P, P, PP, PP, P, P, P, I64, P, ctypes.POINTER(TailParams), P, P, P,
                                  P]
    L.spoly_path_tail.restype = ctypes.c_int
    _lib = L
    return L


def _check(st: int, what: str):
    if st != SPOLY_OK:
        msg = load_library().spoly_status_str(st).decode()
        raise SpolyError(f"{what}: {msg} ({st})")


def default_params() -> Params:
    p = Params()
    load_library().spoly_default_params(ctypes.byref(p))
    return p


def tt_default_params() -> Params:
    p = Params()
    load_library().spoly_tt_default_params(ctypes.byref(p))
    return p


def _ptr(t: torch.Tensor | None):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class DeviceMesh:
    """SoA mesh resident on the GPU (float64 positions / normals, int32 indices)."""

    def __init__(self, P: np.ndarray, N: np.ndarray, tri: np.ndarray, device="cuda"):
        P = np.asarray(P, dtype=np.float64)
        N = np.asarray(N, dtype=np.float64)
        self.cols = [torch.from_numpy(np.ascontiguousarray(P[:, k])).to(device) for k in range(3)]
        self.cols += [torch.from_numpy(np.ascontiguousarray(N[:, k])).to(device) for k in range(3)]
        self.tri = torch.from_numpy(np.ascontiguousarray(tri, dtype=np.int32).ravel()).to(device)
        self.n_vertices = int(P.shape[0])
        self.n_tris = int(len(self.tri) // 3)
        self.c = Mesh(*[c.data_ptr() for c in self.cols], self.tri.data_ptr(), self.n_vertices, self.n_tris)


class DevicePoints:
    def __init__(self, X: np.ndarray, device="cuda"):
        X = np.asarray(X, dtype=np.float64).reshape(-1, 3)
        self.cols = [torch.from_numpy(np.ascontiguousarray(X[:, k])).to(device) for k in range(3)]
        self.n = int(X.shape[0])
        self.c = Points(*[c.data_ptr() for c in self.cols], self.n)


class Context:
    """A spoly_ctx on one device."""

    def __init__(self, device: int = 0):
        L = load_library()
        torch.cuda.set_device(device)
        h = ctypes.c_void_p()
        _check(L.spoly_ctx_create(ctypes.byref(h), device), "spoly_ctx_create")
        self.h = h
        self.device = device

    def close(self):
        if self.h:
            load_library().spoly_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- normal-cone cull
    def cull_1bounce(self, mesh: DeviceMesh, x0s: DevicePoints, x2s: DevicePoints, eta0=1.0, eta1=1.0,
                     margin=1e-3, capacity: int | None = None):
        """Returns int32 device tensors (q_x0, q_x2, q_tri) of the kept triples."""
        L = load_library()
        total = x0s.n * x2s.n * mesh.n_tris
        cap = capacity if capacity is not None else min(total, 1 << 24)
        while True:
            qx0 = torch.empty(cap, dtype=torch.int32, device="cuda")
            qx2 = torch.empty(cap, dtype=torch.int32, device="cuda")
            qt = torch.empty(cap, dtype=torch.int32, device="cuda")
            cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
            _check(L.spoly_cull_1bounce(self.h, ctypes.byref(mesh.c), ctypes.byref(x0s.c), ctypes.byref(x2s.c),
                                        eta0, eta1, margin, _ptr(qx0), _ptr(qx2), _ptr(qt), cap, _ptr(cnt),
                                        _stream()), "spoly_cull_1bounce")
            n = int(cnt.item())
            if n <= cap:
                return qx0[:n], qx2[:n], qt[:n]
            cap = n

    def stage_times(self) -> list:
        """Kernel durations (ms) of the last spoly_solve_1bounce call made with
        SPOLY_FLAG_STAGE_TIMES (waits for it)."""
        buf = (ctypes.c_float * 8)()
        n = load_library().spoly_stage_times(self.h, buf, 8)
        if n < 0:
            raise SpolyError("spoly_stage_times failed")
        return [float(buf[i]) for i in range(n)]

    # ---------------------------------------------------------------- solve
    def solve_1bounce(self, mesh: DeviceMesh, x0s: DevicePoints, x2s: DevicePoints, q_x0: torch.Tensor,
                      q_x2: torch.Tensor, q_tri: torch.Tensor, event: str, eta0=1.0, eta1=1.0,
                      precision: int = SPOLY_FP64, params: Params | None = None, capacity: int | None = None,
                      counters: torch.Tensor | None = None, diag: torch.Tensor | None = None,
                      out: torch.Tensor | None = None, out_count: torch.Tensor | None = None, sync: bool = True):
        """Enqueue the solve.  With sync=True returns the solutions as a numpy
        structured array (SOLUTION_DTYPE), re-running once with a larger buffer
        on overflow."""
        L = load_library()
        nq = int(q_tri.numel())
        prm = params or default_params()
        cap = capacity if capacity is not None else max(1024, nq // 4)
        ev = SPOLY_T if event == "T" else SPOLY_R
        while True:
            buf = out if out is not None else torch.empty(cap * SOLUTION_DTYPE.itemsize, dtype=torch.uint8,
                                                          device="cuda")
            cnt = out_count if out_count is not None else torch.zeros(1, dtype=torch.int64, device="cuda")
            if out_count is not None:
                cnt.zero_()
            _check(L.spoly_solve_1bounce(self.h, ctypes.byref(mesh.c), ctypes.byref(x0s.c), ctypes.byref(x2s.c),
                                         _ptr(q_x0), _ptr(q_x2), _ptr(q_tri), nq, ev, eta0, eta1, precision,
                                         ctypes.byref(prm), _ptr(buf), buf.numel() // SOLUTION_DTYPE.itemsize,
                                         _ptr(cnt), _ptr(counters), _ptr(diag), _stream()), "spoly_solve_1bounce")
            if not sync:
                return buf, cnt
            n = int(cnt.item())
            capn = buf.numel() // SOLUTION_DTYPE.itemsize
            if n <= capn:
                host = buf[: n * SOLUTION_DTYPE.itemsize].cpu().numpy()
                return host.view(SOLUTION_DTYPE)
            if out is not None:
                raise SpolyError(f"output capacity {capn} < {n} solutions")
            cap = n


def _host_doubles(vals):
    arr = (ctypes.c_double * len(vals))(*[float(v) for v in vals])
    return arr


def _cull_2bounce(self, mesh: DeviceMesh, x0s: DevicePoints, x3s: DevicePoints, eta=(1.0, 1.5, 1.0),
                  margin=1e-3, capacity: int | None = None):
    """Returns int32 device tensors (q_x0, q_x3, q_tris [n,2]) of the kept tuples."""
    L = load_library()
    cap = capacity if capacity is not None else 1 << 22
    e = _host_doubles(eta)
    while True:
        q0 = torch.empty(cap, dtype=torch.int32, device="cuda")
        q3 = torch.empty(cap, dtype=torch.int32, device="cuda")
        t1 = torch.empty(cap, dtype=torch.int32, device="cuda")
        t2 = torch.empty(cap, dtype=torch.int32, device="cuda")
        cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
        _check(L.spoly_cull_2bounce(self.h, ctypes.byref(mesh.c), ctypes.byref(x0s.c), ctypes.byref(x3s.c), e,
                                    margin, _ptr(q0), _ptr(q3), _ptr(t1), _ptr(t2), cap, _ptr(cnt), _stream()),
               "spoly_cull_2bounce")
        n = int(cnt.item())
        if n <= cap:
            return q0[:n], q3[:n], torch.stack([t1[:n], t2[:n]], 1).contiguous()
        cap = n


def _solve_2bounce(self, mesh: DeviceMesh, x0s: DevicePoints, x3s: DevicePoints, q_x0: torch.Tensor,
                   q_x3: torch.Tensor, q_tris: torch.Tensor, eta=(1.0, 1.5, 1.0), params: Params | None = None,
                   sqrt_table=None, capacity: int | None = None, counters: torch.Tensor | None = None,
                   diag: torch.Tensor | None = None, sync: bool = True, out=None, out_count=None, chain: str = "TT"):
    """Chain x0 -> T1 -> T2 -> x3 with the events `chain` ("RR", "RT", "TR",
    "TT": reflection or refraction at T1, then at T2)."""
    L = load_library()
    nq = int(q_x0.numel())
    prm = params or tt_default_params()
    if len(chain) != 2 or set(chain) - {"R", "T"}:
        raise SpolyError(f"chain must be two of R/T, got {chain!r}")
    chain = (ctypes.c_int * 2)(*(SPOLY_R if c == "R" else SPOLY_T for c in chain))
    e = _host_doubles(eta)
    tb = _host_doubles(sqrt_table) if sqrt_table is not None else None
    cap = capacity if capacity is not None else max(1024, nq // 8)
    while True:
        buf = out if out is not None else torch.empty(cap * SOLUTION_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
        cnt = out_count if out_count is not None else torch.zeros(1, dtype=torch.int64, device="cuda")
        if out_count is not None:
            cnt.zero_()
        _check(L.spoly_solve_nbounce(self.h, ctypes.byref(mesh.c), 2, chain, e, ctypes.byref(x0s.c),
                                     ctypes.byref(x3s.c), _ptr(q_x0), _ptr(q_x3), _ptr(q_tris), nq, SPOLY_FP64,
                                     ctypes.byref(prm), tb, _ptr(buf), buf.numel() // SOLUTION_DTYPE.itemsize,
                                     _ptr(cnt), _ptr(counters), _ptr(diag), _stream()), "spoly_solve_nbounce")
        if not sync:
            return buf, cnt
        n = int(cnt.item())
        capn = buf.numel() // SOLUTION_DTYPE.itemsize
        if n <= capn:
            return buf[: n * SOLUTION_DTYPE.itemsize].cpu().numpy().view(SOLUTION_DTYPE)
        if out is not None:
            raise SpolyError(f"output capacity {capn} < {n} solutions")
        cap = n


def _pruner_features(self, mesh, x0s, x3s, q_x0, q_x3, q_tris):
    n = int(q_x0.numel())
    out = torch.empty(n * 48, dtype=torch.float32, device="cuda")
    _check(load_library().spoly_pruner_features(self.h, ctypes.byref(mesh.c), ctypes.byref(x0s.c), ctypes.byref(x3s.c),
                                                _ptr(q_x0), _ptr(q_x3), _ptr(q_tris), n, _ptr(out), _stream()),
           "spoly_pruner_features")
    return out.view(n, 48)


def _pruner_fwd_bwd(self, mesh, x0s, x3s, q_x0, q_x3, q_tris, labels, pos_weight, params, grads, loss):
    n = int(q_x0.numel())
    _check(load_library().spoly_pruner_fwd_bwd(self.h, ctypes.byref(mesh.c), ctypes.byref(x0s.c), ctypes.byref(x3s.c),
                                               _ptr(q_x0), _ptr(q_x3), _ptr(q_tris), n, _ptr(labels),
                                               float(pos_weight), _ptr(params), _ptr(grads), _ptr(loss), _stream()),
           "spoly_pruner_fwd_bwd")


def _pruner_step(self, params, grads, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    _check(load_library().spoly_pruner_step(self.h, _ptr(params), _ptr(grads), _ptr(m), _ptr(v), int(step),
                                            float(lr), float(b1), float(b2), float(eps), _stream()),
           "spoly_pruner_step")


def _prune_score(self, mesh, x0s, x3s, q_x0, q_x3, q_tris, params, threshold, scores=None, keep=None,
                 keep_count=None):
    n = int(q_x0.numel())
    kp = keep if keep is not None else torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
    kc = keep_count if keep_count is not None else torch.zeros(1, dtype=torch.int64, device="cuda")
    _check(load_library().spoly_prune_score(self.h, ctypes.byref(mesh.c), ctypes.byref(x0s.c), ctypes.byref(x3s.c),
                                            _ptr(q_x0), _ptr(q_x3), _ptr(q_tris), n, _ptr(params), float(threshold),
                                            _ptr(scores), _ptr(kp), kp.numel(), _ptr(kc), _stream()),
           "spoly_prune_score")
    return kp, kc


def _solve_mixed(self, mesh1, x0s1, x2s1, q1_x0, q1_x2, q1_tri, event, eta0, eta1, mesh2, x0s2, x3s2, q2_x0,
                 q2_x3, q2_tris, eta2=(1.0, 1.5, 1.0), precision=SPOLY_FP32_POLISH64, params=None, shape=None,
                 out=None, out_count=None, queue=None, sync=True, capacity=None):
    """One persistent launch over both problems; queries of problem 2 are offset
    by the number of problem-1 queries.  With sync=False the caller owns (and
    zeroes) `queue` and `out_count`, e.g. inside a captured graph."""
    L = load_library()
    n1, n2 = int(q1_tri.numel()), int(q2_x0.numel())
    prm = params or default_params()
    shp = shape or MixedShape(2, 256, 0, 0)
    e2 = _host_doubles(eta2)
    ev = SPOLY_T if event == "T" else SPOLY_R
    cap = capacity if capacity is not None else max(1024, (n1 + n2) // 4)
    while True:
        buf = out if out is not None else torch.empty(cap * SOLUTION_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
        cnt = out_count if out_count is not None else torch.zeros(1, dtype=torch.int64, device="cuda")
        qq = queue if queue is not None else torch.zeros(1, dtype=torch.int64, device="cuda")
        if sync:
            cnt.zero_()
            qq.zero_()
        _check(L.spoly_solve_mixed(self.h, ctypes.byref(mesh1.c), ctypes.byref(x0s1.c), ctypes.byref(x2s1.c),
                                   _ptr(q1_x0), _ptr(q1_x2), _ptr(q1_tri), n1, ev, eta0, eta1, ctypes.byref(mesh2.c),
                                   ctypes.byref(x0s2.c), ctypes.byref(x3s2.c), _ptr(q2_x0), _ptr(q2_x3),
                                   _ptr(q2_tris), n2, e2, precision, ctypes.byref(prm), ctypes.byref(shp), _ptr(qq),
                                   _ptr(buf), buf.numel() // SOLUTION_DTYPE.itemsize, _ptr(cnt), _stream()),
               "spoly_solve_mixed")
        if not sync:
            return buf, cnt
        n = int(cnt.item())
        capn = buf.numel() // SOLUTION_DTYPE.itemsize
        if n <= capn:
            return buf[: n * SOLUTION_DTYPE.itemsize].cpu().numpy().view(SOLUTION_DTYPE)
        if out is not None:
            raise SpolyError(f"output capacity {capn} < {n} solutions")
        cap = n


class Bvh:
    """Device bounding volume hierarchy of a DeviceMesh (spoly_bvh_build)."""

    def __init__(self, ctx: "Context", mesh: DeviceMesh):
        h = ctypes.c_void_p()
        _check(load_library().spoly_bvh_build(ctx.h, ctypes.byref(mesh.c), ctypes.byref(h), _stream()),
               "spoly_bvh_build")
        self.h = h
        self.mesh = mesh

    def close(self):
        if self.h:
            load_library().spoly_bvh_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def tail_default_params(**kw) -> TailParams:
    p = TailParams()
    load_library().spoly_tail_default_params(ctypes.byref(p))
    for k, v in kw.items():
        if k == "rcv_normal":
            p.rcv_normal = (ctypes.c_double * 3)(*v)
        else:
            setattr(p, k, v)
    return p


def solutions_to_device(sols: np.ndarray) -> torch.Tensor:
    """SOLUTION_DTYPE records as a device byte tensor."""
    b = np.ascontiguousarray(sols, dtype=SOLUTION_DTYPE).view(np.uint8)
    return torch.from_numpy(b.copy()).cuda()


def _path_tail(self, mesh: DeviceMesh, bvh: Bvh, chain: str, eta, x0s: DevicePoints, xls: DevicePoints,
               q_x0: torch.Tensor, q_xl: torch.Tensor, sols: torch.Tensor, n_sols: int | None = None,
               sol_count: torch.Tensor | None = None, params: TailParams | None = None, mask=None, contrib=None,
               image=None):
    """Visibility mask and contribution of solution records `sols` (device
    bytes, SOLUTION_DTYPE) of the chain `chain` ("R", "T", "RR", ... "TT").
    Returns (mask int32, contrib float64, image float64 or None) device tensors
    (allocated when not given; image is accumulated into when given)."""
    L = load_library()
    k = len(chain)
    if k not in (1, 2) or set(chain) - {"R", "T"}:
        raise SpolyError(f"chain must be one or two of R/T, got {chain!r}")
    n = int(n_sols if n_sols is not None else sols.numel() // SOLUTION_DTYPE.itemsize)
    ch = (ctypes.c_int * k)(*(SPOLY_R if c == "R" else SPOLY_T for c in chain))
    e = _host_doubles(eta)
    prm = params or tail_default_params()
    if mask is None:
        mask = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
    if contrib is None:
        contrib = torch.empty(max(n, 1), dtype=torch.float64, device="cuda")
    _check(L.spoly_path_tail(self.h, ctypes.byref(mesh.c), bvh.h, k, ch, e, ctypes.byref(x0s.c), ctypes.byref(xls.c),
                             _ptr(q_x0), _ptr(q_xl), _ptr(sols), n, _ptr(sol_count), ctypes.byref(prm), _ptr(mask),
                             _ptr(contrib), _ptr(image), _stream()), "spoly_path_tail")
    return mask, contrib, image


Context.path_tail = _path_tail
Context.solve_mixed = _solve_mixed
Context.pruner_features = _pruner_features
Context.pruner_fwd_bwd = _pruner_fwd_bwd
Context.pruner_step = _pruner_step
Context.prune_score = _prune_score
Context.cull_2bounce = _cull_2bounce
Context.solve_2bounce = _solve_2bounce


def sort_solutions(s: np.ndarray) -> np.ndarray:
    """Deterministic order: by (query, v, u) of the first vertex."""
    return s[np.lexsort((s["u"][:, 0], s["v"][:, 0], s["query"]))]
