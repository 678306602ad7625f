"""ctypes front end of the exact CPU oracle (test infrastructure only).

The oracle decides, for each candidate pair of closed triangle meshes,
whether the two surfaces share a point (Section 3.2 "Overlap Join", read
with closed sets; see oracle.cpp).  It shares no code with the HIP library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_SO = os.path.join(_HERE, "_oracle.so")
_lock = threading.Lock()
_lib = None

ORACLE_E_ARG = -1
ORACLE_E_DEGENERATE = -3
ORACLE_E_OVERFLOW = -6


class OracleError(RuntimeError):
    def __init__(self, msg: str, code: int = 0):
        super().__init__(msg)
        self.code = code


def build(force: bool = True) -> str:
    """Compile oracle.cpp into _oracle.so with g++ (host code only)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-pthread",
                               _SRC, "-o", tmp])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
                build(force=True)
            lib = ctypes.CDLL(_SO)
            fp = ctypes.POINTER(ctypes.c_float)
            ip = ctypes.POINTER(ctypes.c_int32)
            lp = ctypes.POINTER(ctypes.c_int64)
            lib.oracle_tri_tri.argtypes = [fp, fp]
            lib.oracle_tri_tri.restype = ctypes.c_int
            lib.oracle_orient3d.argtypes = [fp, fp, fp, fp]
            lib.oracle_orient3d.restype = ctypes.c_int
            lib.oracle_join.argtypes = [fp, ip, lp, lp, ctypes.c_int64,
                                        fp, ip, lp, lp, ctypes.c_int64,
                                        ip, ctypes.c_int64, ctypes.POINTER(ctypes.c_uint8),
                                        ctypes.c_int, ctypes.c_int,
                                        ctypes.POINTER(ctypes.c_uint64)]
            lib.oracle_join.restype = ctypes.c_int
            lib.oracle_set_limb_budget.argtypes = [ctypes.c_int]
            lib.oracle_set_limb_budget.restype = ctypes.c_int
            lib.oracle_winding.argtypes = [fp, ip, lp, lp, ctypes.c_int64, ctypes.c_int64, fp, ctypes.c_int,
                                           ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]
            lib.oracle_winding.restype = ctypes.c_int
            lib.oracle_inside_pairs.argtypes = [fp, ip, lp, lp, ctypes.c_int64, fp, ip, lp, lp, ctypes.c_int64,
                                                ip, ctypes.c_int64, ctypes.POINTER(ctypes.c_uint8), ctypes.c_int]
            lib.oracle_inside_pairs.restype = ctypes.c_int
            _lib = lib
    return _lib


def _ptr(a: np.ndarray, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def tri_tri(t, u) -> bool:
    """Exact closed triangle-triangle intersection of two FP32 triangles
    (each 3x3: rows are vertices)."""
    t = np.ascontiguousarray(np.asarray(t, np.float32).reshape(9))
    u = np.ascontiguousarray(np.asarray(u, np.float32).reshape(9))
    r = _load().oracle_tri_tri(_ptr(t, ctypes.c_float), _ptr(u, ctypes.c_float))
    if r < 0:
        raise OracleError("oracle_tri_tri failed with code %d" % r, r)
    return bool(r)


def orient3d(a, b, c, d) -> int:
    """Exact sign of det[b-a, c-a, d-a] for FP32 points."""
    arrs = [np.ascontiguousarray(np.asarray(x, np.float32).reshape(3)) for x in (a, b, c, d)]
    r = _load().oracle_orient3d(*[_ptr(x, ctypes.c_float) for x in arrs])
    if r < -1:
        raise OracleError("oracle_orient3d failed with code %d" % r, r)
    return int(r)


def join(A, B, pairs, mode: int = 1, threads: int = 0, return_tests: bool = False):
    """flags u8[P]: 1 iff mesh A[i] and mesh B[j] share a point, per pair (i, j).

    A, B: objects with verts f32[V,3], faces i32[F,3], vert_off i64[M+1],
    face_off i64[M+1].  mode 0 = all triangle pairs, 1 = exact box
    sweep-and-prune first.  threads 0 = default_threads()."""
    lib = _load()
    if threads <= 0:
        threads = default_threads()
    pairs = np.ascontiguousarray(np.asarray(pairs, np.int32).reshape(-1, 2))
    flags = np.zeros(pairs.shape[0], np.uint8)
    arrs = []
    for S in (A, B):
        arrs.append((np.ascontiguousarray(S.verts, np.float32), np.ascontiguousarray(S.faces, np.int32),
                     np.ascontiguousarray(S.vert_off, np.int64), np.ascontiguousarray(S.face_off, np.int64)))
    ntests = ctypes.c_uint64(0)
    args = []
    for v, f, vo, fo in arrs:
        args += [_ptr(v, ctypes.c_float), _ptr(f, ctypes.c_int32), _ptr(vo, ctypes.c_int64),
                 _ptr(fo, ctypes.c_int64), ctypes.c_int64(vo.shape[0] - 1)]
    r = lib.oracle_join(*args, _ptr(pairs, ctypes.c_int32), ctypes.c_int64(pairs.shape[0]),
                        _ptr(flags, ctypes.c_uint8), ctypes.c_int(mode), ctypes.c_int(threads),
                        ctypes.byref(ntests))
    if r != 0:
        raise OracleError("oracle_join failed with code %d" % r, r)
    return (flags, int(ntests.value)) if return_tests else flags


def _set_args(S):
    v = np.ascontiguousarray(S.verts, np.float32)
    f = np.ascontiguousarray(S.faces, np.int32)
    vo = np.ascontiguousarray(S.vert_off, np.int64)
    fo = np.ascontiguousarray(S.face_off, np.int64)
    return (v, f, vo, fo), [_ptr(v, ctypes.c_float), _ptr(f, ctypes.c_int32), _ptr(vo, ctypes.c_int64),
                            _ptr(fo, ctypes.c_int64), ctypes.c_int64(vo.shape[0] - 1)]


def winding(S, m: int, p, first_dir: int = 0):
    """(winding number, on_surface) of mesh m of set S about the FP32 point p,
    computed exactly by ray crossings along a generic integer direction (the
    first of a fixed list from number first_dir on that meets no edge or
    vertex).  Inside a closed surface with outward faces: 1; outside: 0."""
    keep, args = _set_args(S)
    q = np.ascontiguousarray(np.asarray(p, np.float32).reshape(3))
    w, on = ctypes.c_int32(0), ctypes.c_int32(0)
    r = _load().oracle_winding(*args, ctypes.c_int64(m), _ptr(q, ctypes.c_float), ctypes.c_int(first_dir),
                               ctypes.byref(w), ctypes.byref(on))
    if r != 0:
        raise OracleError("oracle_winding failed with code %d" % r, r)
    return int(w.value), bool(on.value)


def inside_pairs(A, B, pairs, threads: int = 0):
    """u8[P] per pair (i, j): bit 0 = the first vertex of B_j's first face lies
    inside A_i, bit 1 = the first vertex of A_i's first face lies inside B_j,
    bits 2 / 3 = that vertex lies on the other surface."""
    lib = _load()
    pairs = np.ascontiguousarray(np.asarray(pairs, np.int32).reshape(-1, 2))
    bits = np.zeros(pairs.shape[0], np.uint8)
    ka, aa = _set_args(A)
    kb, ab = _set_args(B)
    r = lib.oracle_inside_pairs(*aa, *ab, _ptr(pairs, ctypes.c_int32), ctypes.c_int64(pairs.shape[0]),
                                _ptr(bits, ctypes.c_uint8), ctypes.c_int(threads if threads > 0 else default_threads()))
    if r != 0:
        raise OracleError("oracle_inside_pairs failed with code %d" % r, r)
    return bits


PREDICATES = ("overlap", "contains", "within", "intersection")


def join_predicates(A, B, pairs, threads: int = 0) -> dict:
    """The join predicates per candidate pair (i in A, j in B), u8 flags
    (Sections 3.2-3.4, surface contact read with closed sets):
      overlap      the closed surfaces share a point;
      contains     no shared point and B_j lies inside A_i (a vertex of B_j
                   has non-zero winding number about A_i);
      within       no shared point and A_i lies inside B_j;
      intersection overlap or contains or within.
    For connected closed surfaces that share no point, one vertex decides on
    which side the whole surface lies."""
    cross = join(A, B, pairs, mode=1, threads=threads)
    bits = inside_pairs(A, B, pairs, threads=threads)
    free = cross == 0
    contains = (free & ((bits & 1) != 0)).astype(np.uint8)
    within = (free & ((bits & 2) != 0)).astype(np.uint8)
    return {"overlap": cross, "contains": contains, "within": within,
            "intersection": (cross | contains | within).astype(np.uint8), "inside_bits": bits}


def set_limb_budget(limbs: int) -> int:
    """Test hook: the number of 64-bit limbs an exact integer may use (1..20,
    default 20).  Returns the previous value."""
    r = _load().oracle_set_limb_budget(int(limbs))
    if r < 0:
        raise OracleError("bad limb budget %d" % limbs, r)
    return r


def default_threads() -> int:
    """Threads the oracle uses by default: the cores this process may run
    on, at most 16 (a GPU host's CPU share per GPU), or PIERCE_ORACLE_THREADS."""
    env = os.environ.get("PIERCE_ORACLE_THREADS")
    if env:
        return max(1, int(env))
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def threads_used(threads: int = 0) -> int:
    return threads if threads > 0 else default_threads()
