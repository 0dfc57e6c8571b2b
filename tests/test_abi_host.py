"""Host-side checks of the C ABI (no GPU needed): every entry point declared in
include/spoly.h is exported by libspoly.so, defaults, status strings and the
argument checks that run before any device call."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "spoly.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(spoly_[a-z0-9_]+)\s*\(", txt)))


def _lib():
    import torch  # noqa: F401  (binds the library to torch's HIP runtime)
    from paper_2405_13409_amd import spoly

    if not os.path.exists(spoly.LIB_PATH):
        from paper_2405_13409_amd import build

        build.build()
    return spoly.load_library()


def test_every_declared_symbol_is_exported():
    L = _lib()
    names = _declared()
    assert "spoly_solve_1bounce" in names and "spoly_ctx_create" in names
    for n in names:
        assert hasattr(L, n), n


def test_defaults_and_status_strings():
    from paper_2405_13409_amd import spoly

    p = spoly.default_params()
    assert (p.pieces, p.bisect_iters, p.iso_eps, p.tau, p.polish_iters) == (100, 10, 1e-9, 1e-6, 6)
    L = _lib()
    assert L.spoly_status_str(0) == b"ok"
    assert L.spoly_status_str(1) == b"invalid argument"
    assert L.spoly_status_str(99) == b"unknown status"


def test_invalid_arguments_rejected_on_host():
    from paper_2405_13409_amd import spoly

    L = _lib()
    p = spoly.default_params()
    cnt = ctypes.c_ulonglong(0)
    # null context / mesh
    st = L.spoly_solve_1bounce(None, None, None, None, None, None, None, 0, 0, 1.0, 1.0, 0, ctypes.byref(p), None,
                               0, ctypes.byref(cnt), None, None, None)
    assert st == spoly.SPOLY_E_INVALID_ARG
    st = L.spoly_cull_1bounce(None, None, None, None, 1.0, 1.0, 0.0, None, None, None, 0, ctypes.byref(cnt), None)
    assert st == spoly.SPOLY_E_INVALID_ARG
    st = L.spoly_ctx_create(None, 0)
    assert st == spoly.SPOLY_E_INVALID_ARG


def test_ctx_create_without_device_reports_device_error():
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_2405_13409_amd import spoly

    L = _lib()
    h = ctypes.c_void_p()
    assert L.spoly_ctx_create(ctypes.byref(h), 0) == spoly.SPOLY_E_DEVICE


def test_noalloc_rejects_oversize_and_bad_args_on_host():
    """The no-allocation one-vertex entry point checks its arguments and its
    workspace limit before touching the device."""
    from paper_2405_13409_amd import spoly

    L = _lib()
    p = spoly.default_params()
    cnt = ctypes.c_ulonglong(0)
    st = L.spoly_solve_1bounce_noalloc(None, None, None, None, None, None, 0, 0, 1.0, 1.0, 0, ctypes.byref(p),
                                       None, 0, ctypes.byref(cnt), None, None, None)
    assert st == spoly.SPOLY_E_INVALID_ARG
    # well-formed (never dereferenced) pointers, one query over each limit
    dummy = (ctypes.c_double * 4)()
    ids = (ctypes.c_int32 * 4)()
    addr = ctypes.cast(dummy, ctypes.c_void_p).value
    mesh = spoly.Mesh(addr, addr, addr, addr, addr, addr, ctypes.cast(ids, ctypes.c_void_p).value, 3, 1)
    pts = spoly.Points(addr, addr, addr, 1)
    q = ctypes.cast(ids, ctypes.c_void_p)
    for ev, lim in ((spoly.SPOLY_R, 2000000), (spoly.SPOLY_T, 450000)):
        st = L.spoly_solve_1bounce_noalloc(ctypes.byref(mesh), ctypes.byref(pts), ctypes.byref(pts), q, q, q,
                                           lim + 1, ev, 1.0, 1.0, 0, ctypes.byref(p), None, 0, ctypes.byref(cnt),
                                           None, None, None)
        assert st == spoly.SPOLY_E_CAPACITY


def test_tail_entry_points_on_host():
    """The path-phase tail's defaults and its argument checks before any
    device call; a null hierarchy handle is ignored by the destroy call."""
    from paper_2405_13409_amd import spoly

    L = _lib()
    p = spoly.tail_default_params()
    assert (p.intensity, p.reflectance, p.t_eps, tuple(p.rcv_normal)) == (1.0, 1.0, 1e-6, (0.0, 0.0, 0.0))
    L.spoly_bvh_destroy(None)
    h = ctypes.c_void_p()
    assert L.spoly_bvh_build(None, None, ctypes.byref(h), None) == spoly.SPOLY_E_INVALID_ARG
    chain = (ctypes.c_int * 1)(spoly.SPOLY_R)
    eta = (ctypes.c_double * 2)(1.0, 1.0)
    st = L.spoly_path_tail(None, None, None, 1, chain, eta, None, None, None, None, None, 0, None, ctypes.byref(p),
                           None, None, None, None)
    assert st == spoly.SPOLY_E_INVALID_ARG


def test_flag_bits():
    from paper_2405_13409_amd import spoly

    bits = (spoly.SPOLY_FLAG_FORCE_FP64, spoly.SPOLY_FLAG_STAGE_TIMES, spoly.SPOLY_FLAG_DETERMINISTIC_ORDER)
    assert len(set(bits)) == 3 and all(b & (b - 1) == 0 for b in bits)
    txt = open(os.path.join(ROOT, "include", "spoly.h")).read()
    assert "SPOLY_FLAG_DETERMINISTIC_ORDER (1u << 3)" in txt
