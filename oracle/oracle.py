"""ctypes front end of the C oracle (``oracle/ecmd_oracle.c``).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg use it.  It shares no code with the HIP path.

``build()`` compiles the C file with the host compiler (no contraction, no
fast math) into ``oracle/_build/libecmd_oracle.so``.
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ecmd_oracle.c")
LIB = os.path.join(HERE, "_build", "libecmd_oracle.so")
CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-std=gnu11", "-shared", "-fPIC"]

OK, EINVAL, ENOMEM, EBUDGET = 0, -1, -2, -4


def build(force: bool = True) -> str:
    os.makedirs(os.path.dirname(LIB), exist_ok=True)
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.run(["cc", *CFLAGS, SRC, "-o", tmp, "-lm"], check=True)
        os.replace(tmp, LIB)
    return LIB


class OrcResult(C.Structure):
    _fields_ = [
        ("status", C.c_int32), ("j_star", C.c_uint32), ("L", C.c_uint32),
        ("d_hat", C.c_float), ("contrast", C.c_double), ("d_end", C.c_double),
        ("gap", C.c_double), ("nodes_expanded", C.c_int64), ("nodes_pruned", C.c_int64),
        ("point_evals", C.c_int64), ("bound_evals", C.c_int64),
        ("K_lo", C.c_uint64), ("K_hi", C.c_int64),
    ]


@dataclass
class BnbResult:
    status: int
    j_star: int
    L: int
    d_hat: float
    K: int
    contrast: float
    d_end: float
    gap: float
    nodes_expanded: int
    nodes_pruned: int
    point_evals: int
    bound_evals: int


_lib = None
_f32p = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
_u64p = np.ctypeslib.ndpointer(np.uint64, flags="C_CONTIGUOUS")
_u32p = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
_u16p = np.ctypeslib.ndpointer(np.uint16, flags="C_CONTIGUOUS")
_i8p = np.ctypeslib.ndpointer(np.int8, flags="C_CONTIGUOUS")


def _bind(path: str):
    L = C.CDLL(path)
    ev = [_f32p, _f32p, _f32p, C.c_int64, C.c_int, C.c_int, C.c_float, C.c_float, C.c_float]
    L.orc_depth.argtypes = [C.c_float, C.c_float, C.c_float]
    L.orc_depth.restype = C.c_int
    L.orc_grid_d.argtypes = [C.c_float, C.c_float, C.c_int, C.c_int64]
    L.orc_grid_d.restype = C.c_float
    L.orc_rate.argtypes = [C.c_float, C.c_float]
    L.orc_rate.restype = C.c_float
    L.orc_pixels.argtypes = ev + [C.c_float, _i32p]
    L.orc_pixels.restype = None
    L.orc_point.argtypes = ev + [C.c_float, C.POINTER(C.c_uint64), C.POINTER(C.c_int64), C.c_void_p]
    L.orc_point.restype = C.c_int
    L.orc_bound.argtypes = ev + [C.c_float, C.c_float, C.POINTER(C.c_uint64),
                                 C.POINTER(C.c_int64), C.c_void_p]
    L.orc_bound.restype = C.c_int
    L.orc_bnb.argtypes = ev + [C.c_float, C.c_float, C.c_float, C.c_double, C.c_int64,
                               C.POINTER(OrcResult)]
    L.orc_bnb.restype = C.c_int
    L.orc_bnb64.argtypes = ev + [C.c_float, C.c_float, C.c_float, C.c_double, C.c_int64,
                                 C.POINTER(OrcResult), C.POINTER(C.c_double)]
    L.orc_bnb64.restype = C.c_int
    L.orc_dense.argtypes = ev + [C.c_float, C.c_float, C.c_float, C.POINTER(OrcResult),
                                 C.c_void_p, C.c_void_p]
    L.orc_dense.restype = C.c_int
    L.orc_point64.argtypes = ev + [C.c_double, C.POINTER(C.c_uint64), C.POINTER(C.c_int64)]
    L.orc_point64.restype = C.c_int
    evp = [_f32p, _f32p, _f32p, _i8p, C.c_int64, C.c_int, C.c_int, C.c_float, C.c_float, C.c_float]
    L.orc_point_pol.argtypes = evp + [C.c_float, C.POINTER(C.c_uint64), C.POINTER(C.c_int64), C.c_void_p]
    L.orc_point_pol.restype = C.c_int
    L.orc_bound_pol.argtypes = evp + [C.c_float, C.c_float, C.POINTER(C.c_uint64), C.POINTER(C.c_int64),
                                      C.c_void_p]
    L.orc_bound_pol.restype = C.c_int
    L.orc_bnb_pol.argtypes = evp + [C.c_float, C.c_float, C.c_float, C.c_double, C.c_int64,
                                    C.POINTER(OrcResult)]
    L.orc_bnb_pol.restype = C.c_int
    L.orc_select.argtypes = [_f64p, C.c_int64, C.c_double, C.c_double, _i64p, _f32p]
    L.orc_select.restype = C.c_int64
    L.orc_downsample.argtypes = [_f32p, _f32p, C.c_int64, C.c_int, C.c_int, C.c_int, _u16p]
    L.orc_downsample.restype = C.c_int
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        _lib = _bind(LIB)
    return _lib


class using:
    """Context manager that points this module at another build of the oracle
    (a copy with a planted mistake, in the tests that show the pins catch it)."""

    def __init__(self, path: str):
        self.path = path

    def __enter__(self):
        global _lib
        self.prev = lib()
        _lib = _bind(self.path)
        return self

    def __exit__(self, *exc):
        global _lib
        _lib = self.prev
        return False


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


class Events:
    """A window's events in the oracle's terms: positions, offsets from the
    window start, the window length tau, sensor size and FOE, and optionally
    the polarities (int8, > 0 positive) for the polarity-aware contrast."""

    def __init__(self, x, y, t_rel, tau, W, H, foe, p=None):
        self.x, self.y, self.t = _f32(x), _f32(y), _f32(t_rel)
        self.tau = float(np.float32(tau))
        self.W, self.H = int(W), int(H)
        self.cx, self.cy = float(np.float32(foe[0])), float(np.float32(foe[1]))
        self.n = int(self.x.shape[0])
        self.p = None if p is None else np.ascontiguousarray(p, dtype=np.int8)

    @classmethod
    def of_window(cls, w, polarity: bool = False):
        s = w.spec
        return cls(w.x, w.y, w.t_rel, s.tau, s.width, s.height, s.foe, w.p if polarity else None)

    def _evp(self):
        assert self.p is not None, "no polarities"
        return (self.x, self.y, self.t, self.p, self.n, self.W, self.H, self.cx, self.cy, self.tau)

    @property
    def M(self) -> int:
        return self.W * self.H

    def _ev(self):
        return (self.x, self.y, self.t, self.n, self.W, self.H, self.cx, self.cy, self.tau)


def depth(d_lo, d_hi, eps) -> int:
    return lib().orc_depth(d_lo, d_hi, eps)


def grid_d(d_lo, d_hi, L, j) -> float:
    return lib().orc_grid_d(d_lo, d_hi, L, int(j))


def rate(d, tau) -> float:
    return lib().orc_rate(d, tau)


def pixels(ev: Events, d: float) -> np.ndarray:
    out = np.empty(ev.n, np.int32)
    lib().orc_pixels(*ev._ev(), d, out)
    return out


def point(ev: Events, d: float, want_image: bool = False):
    S, N = C.c_uint64(), C.c_int64()
    img = np.zeros(ev.M, np.uint32) if want_image else None
    rc = lib().orc_point(*ev._ev(), d, C.byref(S), C.byref(N),
                         img.ctypes.data if want_image else None)
    assert rc == OK, rc
    return (S.value, N.value, img) if want_image else (S.value, N.value)


def bound(ev: Events, d_a: float, d_b: float, want_image: bool = False):
    S, N = C.c_uint64(), C.c_int64()
    img = np.zeros(ev.M, np.uint32) if want_image else None
    rc = lib().orc_bound(*ev._ev(), d_a, d_b, C.byref(S), C.byref(N),
                         img.ctypes.data if want_image else None)
    assert rc == OK, rc
    return (S.value, N.value, img) if want_image else (S.value, N.value)


def key(M: int, S: int, N: int) -> int:
    """Exact contrast key K = M*S - N^2 (= M^2 * contrast)."""
    return int(M) * int(S) - int(N) * int(N)


def _res(r: OrcResult) -> BnbResult:
    K = (int(r.K_hi) << 64) | int(r.K_lo)
    return BnbResult(int(r.status), int(r.j_star), int(r.L), float(r.d_hat), K,
                     float(r.contrast), float(r.d_end), float(r.gap), int(r.nodes_expanded),
                     int(r.nodes_pruned), int(r.point_evals), int(r.bound_evals))


def bnb(ev: Events, d_lo: float, d_hi: float, eps: float, gamma: float = 0.0,
        max_nodes: int = 0) -> BnbResult:
    r = OrcResult()
    lib().orc_bnb(*ev._ev(), d_lo, d_hi, eps, gamma, max_nodes, C.byref(r))
    return _res(r)


def bnb64(ev: Events, d_lo: float, d_hi: float, eps: float, gamma: float = 0.0,
          max_nodes: int = 0):
    r = OrcResult()
    d64 = C.c_double()
    lib().orc_bnb64(*ev._ev(), d_lo, d_hi, eps, gamma, max_nodes, C.byref(r), C.byref(d64))
    return _res(r), d64.value


def dense(ev: Events, d_lo: float, d_hi: float, eps: float, want_all: bool = False):
    r = OrcResult()
    if want_all:
        L = depth(d_lo, d_hi, eps)
        S = np.zeros((1 << L) + 1, np.uint64)
        N = np.zeros((1 << L) + 1, np.int64)
        lib().orc_dense(*ev._ev(), d_lo, d_hi, eps, C.byref(r), S.ctypes.data, N.ctypes.data)
        return _res(r), S, N
    lib().orc_dense(*ev._ev(), d_lo, d_hi, eps, C.byref(r), None, None)
    return _res(r)


def point64(ev: Events, d: float):
    S, N = C.c_uint64(), C.c_int64()
    rc = lib().orc_point64(*ev._ev(), float(d), C.byref(S), C.byref(N))
    assert rc == OK, rc
    return S.value, N.value


def select(t: np.ndarray, t0: float, t1: float):
    t = np.ascontiguousarray(t, np.float64)
    idx = np.empty(t.shape[0], np.int64)
    tr = np.empty(t.shape[0], np.float32)
    m = lib().orc_select(t, t.shape[0], t0, t1, idx, tr)
    return idx[:m], tr[:m]


def downsample(x, y, W: int, H: int, G: int = 64) -> np.ndarray:
    out = np.empty(G * G, np.uint16)
    rc = lib().orc_downsample(_f32(x), _f32(y), int(np.asarray(x).shape[0]), W, H, G, out)
    assert rc == OK
    return out.reshape(G, G)


# ------------------------------------------------- polarity-aware contrast

def point_pol(ev: Events, d: float, want_image: bool = False):
    """(S, N) over the two polarity images; the key uses 2M cells."""
    S, N = C.c_uint64(), C.c_int64()
    img = np.zeros(2 * ev.M, np.uint32) if want_image else None
    rc = lib().orc_point_pol(*ev._evp(), d, C.byref(S), C.byref(N), img.ctypes.data if want_image else None)
    assert rc == OK, rc
    return (S.value, N.value, img) if want_image else (S.value, N.value)


def bound_pol(ev: Events, d_a: float, d_b: float, want_image: bool = False):
    S, N = C.c_uint64(), C.c_int64()
    img = np.zeros(2 * ev.M, np.uint32) if want_image else None
    rc = lib().orc_bound_pol(*ev._evp(), d_a, d_b, C.byref(S), C.byref(N),
                             img.ctypes.data if want_image else None)
    assert rc == OK, rc
    return (S.value, N.value, img) if want_image else (S.value, N.value)


def bnb_pol(ev: Events, d_lo: float, d_hi: float, eps: float, gamma: float = 0.0,
            max_nodes: int = 0) -> BnbResult:
    r = OrcResult()
    lib().orc_bnb_pol(*ev._evp(), d_lo, d_hi, eps, gamma, max_nodes, C.byref(r))
    return _res(r)
