"""CPU max-flow oracle -- TEST INFRASTRUCTURE ONLY.

Only the tests, the package smoke check and the benchmark's CPU-baseline leg
use this package.  It wraps the plain C oracle in `oracle.c` (built with gcc
into `liboracle.so` next to it) and shares nothing with the HIP library.

Functions follow the paper's definitions:
  * brute_min_cut      -- F* as the minimum s-t cut (Section 2.1 problem,
                          max-flow min-cut theorem), by enumeration;
  * edmonds_karp       -- shortest augmenting paths (Section 2.2);
  * DynOracle          -- sequential push-relabel with gap and global
                          relabel (Section 2.2), static solve as in
                          Algorithm 1 and batch repair as in Algorithm 5;
  * cert_check         -- flow feasibility + conservation + equal-capacity
                          cut, the certificate of Sections 3.1 and 4.3.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-std=c11", "-fPIC", "-shared", "-Wall", "-Wextra",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def build_native(dest: str) -> str:
    """Compile oracle.c with -O3 -march=native for the machine this runs on
    (the benchmark's CPU baseline builds its own copy where it times it; the
    in-tree library stays portable).  Load it by setting MF_ORACLE_LIB before
    the first call."""
    tmp = dest + ".tmp"
    subprocess.check_call(["gcc", "-O3", "-march=native", "-std=c11", "-fPIC", "-shared", "-o", tmp, _SRC])
    os.replace(tmp, dest)
    return dest


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("MF_ORACLE_LIB")  # a rebuilt variant, used by the mutation tests
        if path is None:
            path = _LIB
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build()
        L = C.CDLL(path)
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C")
        i64p = np.ctypeslib.ndpointer(np.int64, flags="C")
        u8p = np.ctypeslib.ndpointer(np.uint8, flags="C")
        L.or_brute_min_cut.restype = C.c_int64
        L.or_brute_min_cut.argtypes = [C.c_int32, C.c_int64, i32p, i32p, i32p, C.c_int32, C.c_int32]
        L.or_edmonds_karp.restype = C.c_int64
        L.or_edmonds_karp.argtypes = [C.c_int32, C.c_int64, i32p, i32p, i32p, C.c_int32, C.c_int32,
                                      C.c_void_p, C.c_void_p]
        L.og_create.restype = C.c_void_p
        L.og_create.argtypes = [C.c_int32, C.c_int64, i32p, i32p, i32p, C.c_int32, C.c_int32]
        L.og_free.argtypes = [C.c_void_p]
        L.og_num_pairs.restype = C.c_int64
        L.og_num_pairs.argtypes = [C.c_void_p]
        L.og_static.restype = C.c_int64
        L.og_static.argtypes = [C.c_void_p]
        L.og_apply.restype = C.c_int64
        L.og_apply.argtypes = [C.c_void_p, C.c_int64, i32p, i32p, i32p]
        L.og_min_cut.restype = C.c_int64
        L.og_min_cut.argtypes = [C.c_void_p, u8p]
        L.og_initial_labels.argtypes = [C.c_void_p, i32p, i64p]
        L.og_state.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.og_pairs.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.og_stats.argtypes = [C.c_void_p, i64p]
        L.or_cert_check.restype = C.c_int
        L.or_cert_check.argtypes = [C.c_int32, C.c_int64, i32p, i32p, i32p, C.c_int32, C.c_int32,
                                    C.c_void_p, C.c_void_p, C.c_int64, C.c_char_p, C.c_int32]
        _lib = L
    return _lib


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def brute_min_cut(n, src, dst, cap, s, t) -> int:
    """Minimum s-t cut by enumerating all 2**(n-2) source sides (n <= 22)."""
    src, dst, cap = _i32(src), _i32(dst), _i32(cap)
    v = lib().or_brute_min_cut(n, src.size, src, dst, cap, s, t)
    if v < 0:
        raise ValueError("brute force needs 2 <= n <= 22 and s != t")
    return int(v)


def edmonds_karp(n, src, dst, cap, s, t):
    """Returns (value, flow per input edge int64, side uint8 = reachable from s)."""
    src, dst, cap = _i32(src), _i32(dst), _i32(cap)
    flow = np.zeros(src.size, np.int64)
    side = np.zeros(n, np.uint8)
    v = lib().or_edmonds_karp(n, src.size, src, dst, cap, s, t, flow.ctypes.data, side.ctypes.data)
    return int(v), flow, side


def cert_check(n, src, dst, cap, s, t, flow, side, value):
    """Returns (code, message); code 0 means every requested check passed."""
    src, dst, cap = _i32(src), _i32(dst), _i32(cap)
    f = None if flow is None else np.ascontiguousarray(flow, dtype=np.int64)
    sd = None if side is None else np.ascontiguousarray(side, dtype=np.uint8)
    msg = C.create_string_buffer(256)
    rc = lib().or_cert_check(n, src.size, src, dst, cap, s, t,
                             None if f is None else f.ctypes.data,
                             None if sd is None else sd.ctypes.data, int(value), msg, 256)
    return int(rc), msg.value.decode()


class DynOracle:
    """Sequential push-relabel over merged capacities; keeps its residual
    state between calls so that `apply` repairs it as Algorithm 5 does."""

    def __init__(self, n, src, dst, cap, s, t):
        src, dst, cap = _i32(src), _i32(dst), _i32(cap)
        self.n, self.s, self.t = int(n), int(s), int(t)
        self._h = lib().og_create(n, src.size, src, dst, cap, s, t)
        if not self._h:
            raise ValueError("invalid graph for the oracle")

    def close(self):
        if self._h:
            lib().og_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def static(self) -> int:
        return int(lib().og_static(self._h))

    def apply(self, u, v, c) -> int:
        u, v, c = _i32(u), _i32(v), _i32(c)
        val = lib().og_apply(self._h, u.size, u, v, c)
        if val < 0:
            raise ValueError("invalid update batch")
        return int(val)

    def min_cut(self):
        side = np.zeros(self.n, np.uint8)
        c = lib().og_min_cut(self._h, side)
        return side, int(c)

    def initial_labels(self):
        h = np.zeros(self.n, np.int32)
        e = np.zeros(self.n, np.int64)
        lib().og_initial_labels(self._h, h, e)
        return h, e

    def state(self):
        e = np.zeros(self.n, np.int64)
        h = np.zeros(self.n, np.int32)
        lib().og_state(self._h, e.ctypes.data, h.ctypes.data)
        return e, h

    def pairs(self):
        k = int(lib().og_num_pairs(self._h))
        u = np.zeros(k, np.int32)
        v = np.zeros(k, np.int32)
        c = np.zeros(k, np.int64)
        f = np.zeros(k, np.int64)
        lib().og_pairs(self._h, u.ctypes.data, v.ctypes.data, c.ctypes.data, f.ctypes.data)
        return u, v, c, f

    def stats(self):
        out = np.zeros(4, np.int64)
        lib().og_stats(self._h, out)
        return dict(zip(["pushes", "relabels", "gaps", "global_relabels"], out.tolist()))


def max_flow(n, src, dst, cap, s, t) -> int:
    """F* of a graph from scratch (sequential push-relabel)."""
    o = DynOracle(n, src, dst, cap, s, t)
    try:
        return o.static()
    finally:
        o.close()
