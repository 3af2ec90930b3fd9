"""Thin Python binding of ``libecmd.so`` (argument marshalling only).

Every step of the estimator runs in the library's HIP kernels; this module
only converts arrays to pointers.  Arrays may be NumPy (host memory) or
torch tensors on the context's GPU (device memory, ``ECMD_DEVICE_PTR``); a
call uses one kind for all its arrays.  The library must have been built
(``paper_2209_13168_amd/build.py``); importing fails loudly otherwise.
"""

from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, fields
from typing import Optional, Sequence

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "_build", "libecmd.so")

OK, EINVAL, ENOMEM, EDEVICE, EBUDGET, EFRONTIER = 0, -1, -2, -3, -4, -5
SEARCH_EXACT_BOUNDS = 1  # ecmd_search.flags: every child interval gets the exact bound
DEVICE_PTR = 1
CNN_NPARAM = 23361
GRID = 64


class EcmdError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"ecmd error {code}: {msg}")
        self.code = code


class Sensor(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("foe_x", C.c_float), ("foe_y", C.c_float)]


class EventsS(C.Structure):
    _fields_ = [("x", C.c_void_p), ("y", C.c_void_p), ("t", C.c_void_p), ("n", C.c_int64), ("p", C.c_void_p)]


class WindowS(C.Structure):
    _fields_ = [("t0", C.c_double), ("t1", C.c_double)]


class SearchS(C.Structure):
    _fields_ = [("d_lo", C.c_float), ("d_hi", C.c_float), ("eps", C.c_float), ("flags", C.c_uint32),
                ("gamma", C.c_double), ("max_nodes", C.c_int64), ("frontier_batch", C.c_int32),
                ("frontier_capacity", C.c_int32)]


class ResultS(C.Structure):
    _fields_ = [("status", C.c_int32), ("j_star", C.c_uint32), ("L", C.c_uint32), ("d_hat", C.c_float),
                ("contrast", C.c_double), ("d_end", C.c_double), ("gap", C.c_double),
                ("K_lo", C.c_uint64), ("K_hi", C.c_int64), ("n_events", C.c_int64),
                ("nodes_expanded", C.c_int64), ("nodes_pruned", C.c_int64), ("point_evals", C.c_int64),
                ("bound_evals", C.c_int64), ("event_hyp_evals", C.c_int64), ("pixel_updates", C.c_int64),
                ("steps", C.c_int32), ("seeded", C.c_int32), ("bound_certs", C.c_int64)]


class PlanInfo(C.Structure):
    _fields_ = [("L", C.c_int32), ("segments", C.c_int32), ("ntx", C.c_int32), ("nty", C.c_int32),
                ("max_tile_px", C.c_int32), ("tile_budget_px", C.c_int32), ("colcut", C.c_int32 * 65),
                ("rowcut", C.c_int32 * 65), ("eval_threads", C.c_int32)]


class PlanLimitsS(C.Structure):
    _fields_ = [("max_windows", C.c_int32), ("max_steps", C.c_int32), ("max_events", C.c_int64),
                ("max_records", C.c_int64), ("polarity", C.c_int32), ("reserved", C.c_int32)]


class TuningS(C.Structure):
    _fields_ = [("frontier_batch", C.c_int32), ("tile_px", C.c_int32), ("graph", C.c_int32),
                ("group", C.c_int32), ("eval_threads", C.c_int32)]


class ProfileS(C.Structure):
    _fields_ = [("calls", C.c_int64), ("eval_launches", C.c_int64), ("eval_ms", C.c_double),
                ("frontier_launches", C.c_int64), ("frontier_ms", C.c_double), ("prep_ms", C.c_double)]


@dataclass
class Result:
    status: int
    j_star: int
    L: int
    d_hat: float
    K: int
    contrast: float
    d_end: float
    gap: float
    n_events: int
    nodes_expanded: int
    nodes_pruned: int
    point_evals: int
    bound_evals: int
    event_hyp_evals: int
    pixel_updates: int
    steps: int
    seeded: int
    bound_certs: int

    @classmethod
    def of(cls, r: ResultS) -> "Result":
        K = (int(r.K_hi) << 64) | int(r.K_lo)
        vals = {f.name: getattr(r, f.name) for f in fields(cls) if f.name != "K"}
        return cls(K=K, **vals)


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build the HIP library first "
                          "(python paper_2209_13168_amd/build.py)")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, u32, f32 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32, C.c_float
    sig = {
        "ecmd_version": ([], C.c_char_p),
        "ecmd_ctx_create": ([C.POINTER(vp), C.c_int, vp], C.c_int),
        "ecmd_ctx_destroy": ([vp], None),
        "ecmd_last_error": ([vp], C.c_char_p),
        "ecmd_estimate_divergence": ([vp, C.POINTER(Sensor), C.POINTER(EventsS), WindowS,
                                      C.POINTER(SearchS), u32, vp, C.POINTER(ResultS)], C.c_int),
        "ecmd_estimate_divergence_batched": ([vp, C.POINTER(Sensor), vp, vp, vp, vp, vp, i32,
                                              C.POINTER(SearchS), u32, vp, C.POINTER(ResultS)], C.c_int),
        "ecmd_estimate_divergence_batched_polarity": ([vp, C.POINTER(Sensor), vp, vp, vp, vp, vp, vp, i32,
                                                       C.POINTER(SearchS), u32, vp, C.POINTER(ResultS)], C.c_int),
        "ecmd_probe_pixels": ([vp, C.POINTER(Sensor), vp, vp, vp, i64, f32, f32, u32, vp], C.c_int),
        "ecmd_probe_point": ([vp, C.POINTER(Sensor), vp, vp, vp, vp, i64, f32, vp, i32, u32, vp, vp, vp],
                             C.c_int),
        "ecmd_probe_bound": ([vp, C.POINTER(Sensor), vp, vp, vp, vp, i64, f32, f32, f32, vp, vp, i32, u32,
                              vp, vp, vp], C.c_int),
        "ecmd_downsample": ([vp, C.POINTER(Sensor), vp, vp, vp, i32, u32, vp], C.c_int),
        "ecmd_ctx_set_profiling": ([vp, C.c_int], C.c_int),
        "ecmd_plan": ([C.POINTER(Sensor), C.POINTER(SearchS), i32, i64, i32, C.POINTER(PlanInfo)], C.c_int),
        "ecmd_grid_point": ([f32, f32, u32, u32], f32),
        "ecmd_plan_create": ([vp, C.POINTER(Sensor), C.POINTER(SearchS), C.POINTER(PlanLimitsS), C.POINTER(vp)],
                             C.c_int),
        "ecmd_plan_launch": ([vp, vp, vp, vp, vp, vp, vp, i32, vp, vp], C.c_int),
        "ecmd_plan_destroy": ([vp], None),
        "ecmd_estimate_divergence_batched_noalloc": ([vp, C.POINTER(Sensor), C.POINTER(SearchS), vp, vp, vp, vp, vp,
                                                      i32, i64, vp, vp], C.c_int),
        "ecmd_measure_peaks": ([vp, i64, C.POINTER(C.c_double), C.POINTER(C.c_double)], C.c_int),
        "ecmd_ctx_set_tuning": ([vp, C.POINTER(TuningS)], C.c_int),
        "ecmd_ctx_get_tuning": ([vp, C.POINTER(TuningS)], C.c_int),
        "ecmd_autotune": ([vp, C.POINTER(Sensor), vp, vp, vp, vp, vp, i32, C.POINTER(SearchS), u32,
                           C.POINTER(TuningS), C.POINTER(C.c_double)], C.c_int),
        "ecmd_ctx_get_profile": ([vp, C.POINTER(ProfileS), C.c_int], C.c_int),
        "ecmd_estimate_stream": ([vp, C.POINTER(Sensor), C.POINTER(EventsS), C.c_double, C.c_double, i32,
                                  C.POINTER(SearchS), u32, C.POINTER(ResultS)], C.c_int),
        "ecmd_hot_pixel_filter": ([vp, C.POINTER(Sensor), vp, vp, vp, vp, i32, i32, u32, vp, vp, vp, vp], C.c_int),
        "ecmd_resample": ([vp, C.POINTER(Sensor), C.POINTER(Sensor), vp, vp, vp, vp, i32, f32, C.c_uint64, u32,
                           vp, vp, vp, vp], C.c_int),
        "ecmd_cnn_create": ([vp, C.c_uint64, C.POINTER(vp)], C.c_int),
        "ecmd_cnn_destroy": ([vp], None),
        "ecmd_cnn_get_params": ([vp, vp], C.c_int),
        "ecmd_cnn_set_params": ([vp, vp], C.c_int),
        "ecmd_cnn_forward": ([vp, vp, i32, u32, vp], C.c_int),
        "ecmd_cnn_save": ([vp, C.c_char_p], C.c_int),
        "ecmd_cnn_load": ([vp, C.c_char_p], C.c_int),
        "ecmd_cnn_grads": ([vp, vp, vp, i32, u32, vp, vp], C.c_int),
        "ecmd_cnn_train_step": ([vp, vp, vp, i32, f32, u32, vp], C.c_int),
        "ecmd_estimate_divergence_learned": ([vp, vp, C.POINTER(Sensor), vp, vp, vp, vp, vp, i32,
                                              C.POINTER(SearchS), u32, C.POINTER(ResultS)], C.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name, None)
        if fn is None:
            continue
        fn.argtypes = args
        fn.restype = res
    return L


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = _load()
    return _lib


def _is_torch(a) -> bool:
    return type(a).__module__.startswith("torch")


class _Args:
    """Pointer marshalling for one call: all arrays host (NumPy) or all
    device (torch CUDA tensors)."""

    def __init__(self):
        self.keep = []
        self.device = None

    def ptr(self, a, dtype):
        if a is None:
            return None
        if _is_torch(a):
            import torch

            tdt = {np.float32: torch.float32, np.float64: torch.float64, np.int64: torch.int64,
                   np.int32: torch.int32, np.uint64: torch.int64, np.uint32: torch.int32,
                   np.uint16: torch.int16, np.int8: torch.int8}[dtype]
            if a.dtype != tdt or not a.is_contiguous() or not a.is_cuda:
                raise TypeError(f"expected a contiguous CUDA tensor of {tdt}, got {a.dtype} on {a.device}")
            if self.device is False:
                raise TypeError("mixing host and device arrays in one call")
            self.device = True
            self.keep.append(a)
            return a.data_ptr()
        arr = np.ascontiguousarray(a, dtype=dtype)
        if self.device is True:
            raise TypeError("mixing host and device arrays in one call")
        self.device = False
        self.keep.append(arr)
        return arr.ctypes.data

    @property
    def flags(self) -> int:
        return DEVICE_PTR if self.device else 0


def _search(d_lo, d_hi, eps, gamma=0.0, max_nodes=0, frontier_batch=0, frontier_capacity=0,
            exact_bounds=False) -> SearchS:
    return SearchS(float(d_lo), float(d_hi), float(eps), SEARCH_EXACT_BOUNDS if exact_bounds else 0, float(gamma),
                   int(max_nodes), int(frontier_batch), int(frontier_capacity))


def plan(sensor: Sensor, d_lo: float, d_hi: float, eps: float, polarity: bool = False, lds_bytes: int = 0,
         tile_px: int = 0) -> dict:
    """Grid depth and image tiling of a search (host only, no device)."""
    out = PlanInfo()
    rc = lib().ecmd_plan(C.byref(sensor), C.byref(_search(d_lo, d_hi, eps)), 1 if polarity else 0, int(lds_bytes),
                         int(tile_px), C.byref(out))
    if rc != OK:
        raise EcmdError(rc, "invalid plan arguments")
    return {"L": out.L, "segments": out.segments, "ntx": out.ntx, "nty": out.nty, "max_tile_px": out.max_tile_px,
            "tile_budget_px": out.tile_budget_px, "colcut": list(out.colcut[:out.ntx + 1]),
            "rowcut": list(out.rowcut[:out.nty + 1]), "eval_threads": out.eval_threads}


def grid_point(d_lo: float, d_hi: float, L: int, j: int) -> float:
    return float(lib().ecmd_grid_point(float(d_lo), float(d_hi), int(L), int(j)))


class Context:
    """A library context on one GPU, ordered on a HIP stream (default: the
    current torch stream of that device, when torch is loaded)."""

    def __init__(self, device: int = 0, stream: Optional[int] = None):
        if stream is None:
            try:
                import torch

                if torch.cuda.is_available():
                    stream = torch.cuda.current_stream(device).cuda_stream
            except ImportError:  # pragma: no cover
                stream = None
        h = C.c_void_p()
        rc = lib().ecmd_ctx_create(C.byref(h), int(device), C.c_void_p(stream or 0))
        if rc != OK:
            raise EcmdError(rc, "ecmd_ctx_create failed (no usable HIP device?)")
        self.h = h
        self.device = device

    def close(self):
        if getattr(self, "h", None):
            lib().ecmd_ctx_destroy(self.h)
            self.h = None

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _check(self, rc: int, allow=()):
        if rc != OK and rc not in allow:
            raise EcmdError(rc, lib().ecmd_last_error(self.h).decode())
        return rc

    def last_error(self) -> str:
        return lib().ecmd_last_error(self.h).decode()

    def set_tuning(self, frontier_batch: int = 0, tile_px: int = 0, graph: bool = False, group: int = 0,
                   eval_threads: int = 0):
        t = TuningS(int(frontier_batch), int(tile_px), 1 if graph else 0, int(group), int(eval_threads))
        self._check(lib().ecmd_ctx_set_tuning(self.h, C.byref(t)))

    def tuning(self) -> dict:
        t = TuningS()
        self._check(lib().ecmd_ctx_get_tuning(self.h, C.byref(t)))
        return {"frontier_batch": t.frontier_batch, "tile_px": t.tile_px, "graph": bool(t.graph), "group": t.group,
                "eval_threads": t.eval_threads}

    def autotune(self, sensor: Sensor, x, y, t_rel, offsets, tau, d_lo: float, d_hi: float, eps: float,
                 cache: Optional[str] = None) -> dict:
        """Pick the fastest launch tuning for this kind of batch (kept in the
        context).  With a cache file (JSON; default $ECMD_TUNE_CACHE) the
        result is stored under a key of sensor size, batch size and mean
        event count, and reused on later calls."""
        import json

        cache = cache or os.environ.get("ECMD_TUNE_CACHE")
        B = int(tau.shape[0])
        n_mean = int(offsets[-1] - offsets[0]) // max(B, 1)
        key = f"{sensor.width}x{sensor.height}/B{1 << max(B - 1, 0).bit_length()}/N{1 << max(n_mean - 1, 0).bit_length()}"
        if cache and os.path.exists(cache):
            with open(cache) as f:
                known = json.load(f)
            if key in known:
                self.set_tuning(**{k: known[key].get(k, 0)
                                   for k in ("frontier_batch", "tile_px", "graph", "group", "eval_threads")})
                return dict(known[key], cached=True)
        a = _Args()
        px, py, pt = a.ptr(x, np.float32), a.ptr(y, np.float32), a.ptr(t_rel, np.float32)
        po, ptau = a.ptr(offsets, np.int64), a.ptr(tau, np.float32)
        sp = _search(d_lo, d_hi, eps)
        best = TuningS()
        ms = C.c_double()
        self._check(lib().ecmd_autotune(self.h, C.byref(sensor), px, py, pt, po, ptau, B, C.byref(sp), a.flags,
                                        C.byref(best), C.byref(ms)))
        out = {"frontier_batch": best.frontier_batch, "tile_px": best.tile_px, "graph": bool(best.graph),
               "group": best.group, "eval_threads": best.eval_threads, "ms": ms.value}
        if cache:
            known = {}
            if os.path.exists(cache):
                with open(cache) as f:
                    known = json.load(f)
            known[key] = out
            with open(cache, "w") as f:
                json.dump(known, f, indent=1, sort_keys=True)
        return dict(out, cached=False)

    def set_profiling(self, enable: bool = True):
        self._check(lib().ecmd_ctx_set_profiling(self.h, 1 if enable else 0))

    def profile(self, reset: bool = False) -> dict:
        p = ProfileS()
        self._check(lib().ecmd_ctx_get_profile(self.h, C.byref(p), 1 if reset else 0))
        return {f[0]: getattr(p, f[0]) for f in ProfileS._fields_}

    def measure_peaks(self, hbm_bytes: int = 0) -> dict:
        """Measured LDS-atomic rate (lane ops/s) and HBM read bandwidth (B/s)."""
        lds, hbm = C.c_double(), C.c_double()
        self._check(lib().ecmd_measure_peaks(self.h, int(hbm_bytes), C.byref(lds), C.byref(hbm)))
        return {"lds_atomics_per_s": lds.value, "hbm_read_bytes_per_s": hbm.value}

    # ---------------------------------------------------------- estimation
    def estimate(self, sensor: Sensor, x, y, t, t0: float, t1: float, d_lo: float, d_hi: float, eps: float,
                 gamma: float = 0.0, max_nodes: int = 0, frontier_batch: int = 0, frontier_capacity: int = 0,
                 d_seed: Optional[float] = None, polarity=None, exact_bounds: bool = False) -> Result:
        """One window [t0, t1] of a stream; polarity (int8, optional) selects
        the polarity-aware contrast."""
        a = _Args()
        n = int(x.shape[0])
        ev = EventsS(a.ptr(x, np.float32), a.ptr(y, np.float32), a.ptr(t, np.float64), n,
                     a.ptr(polarity, np.int8))
        sp = _search(d_lo, d_hi, eps, gamma, max_nodes, frontier_batch, frontier_capacity, exact_bounds)
        seed = C.c_float(d_seed) if d_seed is not None else None
        out = ResultS()
        rc = lib().ecmd_estimate_divergence(self.h, C.byref(sensor), C.byref(ev), WindowS(t0, t1), C.byref(sp),
                                            a.flags, C.byref(seed) if seed is not None else None, C.byref(out))
        self._check(rc, allow=(EBUDGET, EFRONTIER))
        return Result.of(out)

    def estimate_batched(self, sensor: Sensor, x, y, t_rel, offsets, tau, d_lo: float, d_hi: float,
                         eps: float, gamma: float = 0.0, max_nodes: int = 0, frontier_batch: int = 0,
                         frontier_capacity: int = 0, d_seeds=None, polarity=None, exact_bounds: bool = False) -> list:
        """B windows in one call; polarity (int8 per event, optional) selects
        the polarity-aware contrast."""
        a = _Args()
        B = int(tau.shape[0])
        px, py, pt = a.ptr(x, np.float32), a.ptr(y, np.float32), a.ptr(t_rel, np.float32)
        po, ptau = a.ptr(offsets, np.int64), a.ptr(tau, np.float32)
        ps = a.ptr(d_seeds, np.float32) if d_seeds is not None else None
        sp = _search(d_lo, d_hi, eps, gamma, max_nodes, frontier_batch, frontier_capacity, exact_bounds)
        out = (ResultS * max(B, 1))()
        if polarity is None:
            rc = lib().ecmd_estimate_divergence_batched(self.h, C.byref(sensor), px, py, pt, po, ptau, B,
                                                        C.byref(sp), a.flags, ps, out)
        else:
            pp = a.ptr(polarity, np.int8)
            rc = lib().ecmd_estimate_divergence_batched_polarity(self.h, C.byref(sensor), px, py, pt, pp, po, ptau,
                                                                 B, C.byref(sp), a.flags, ps, out)
        self._check(rc, allow=(EBUDGET, EFRONTIER))
        return [Result.of(out[i]) for i in range(B)]

    def batch_plan(self, sensor: Sensor, d_lo: float, d_hi: float, eps: float, max_windows: int, max_events: int,
                   gamma: float = 0.0, max_nodes: int = 0, frontier_batch: int = 0, frontier_capacity: int = 0,
                   max_steps: int = 0, max_records: int = 0, polarity: bool = False,
                   exact_bounds: bool = False) -> "BatchPlan":
        """Device buffers for asynchronous batched searches up to the limits."""
        sp = _search(d_lo, d_hi, eps, gamma, max_nodes, frontier_batch, frontier_capacity, exact_bounds)
        return BatchPlan(self, sensor, sp,
                         PlanLimitsS(int(max_windows), int(max_steps), int(max_events), int(max_records),
                                     1 if polarity else 0, 0))

    def estimate_batched_noalloc(self, sensor: Sensor, x, y, t_rel, offsets, tau, d_lo: float, d_hi: float,
                                 eps: float, max_events: int, out, gamma: float = 0.0, max_nodes: int = 0,
                                 frontier_batch: int = 0, frontier_capacity: int = 0, d_seeds=None,
                                 exact_bounds: bool = False):
        """The batched search on the library's static scratch (no device
        allocation): torch CUDA tensors in, results into ``out`` (a
        ``BatchPlan.result_buffer``) when the stream reaches them."""
        a = _Args()
        B = int(tau.shape[0])
        args = [a.ptr(x, np.float32), a.ptr(y, np.float32), a.ptr(t_rel, np.float32), a.ptr(offsets, np.int64),
                a.ptr(tau, np.float32), B, int(max_events),
                a.ptr(d_seeds, np.float32) if d_seeds is not None else None]
        if not a.device:
            raise TypeError("the allocation-free search takes device arrays")
        if out.numel() < C.sizeof(ResultS) * B:
            raise ValueError("result buffer too small")
        sp = _search(d_lo, d_hi, eps, gamma, max_nodes, frontier_batch, frontier_capacity, exact_bounds)
        rc = lib().ecmd_estimate_divergence_batched_noalloc(self.h, C.byref(sensor), C.byref(sp), *args,
                                                            C.c_void_p(out.data_ptr()))
        self._check(rc)

    # -------------------------------------------------------------- probes
    def probe_pixels(self, sensor: Sensor, x, y, t_rel, tau: float, d: float, out=None):
        a = _Args()
        n = int(x.shape[0])
        px, py, pt = a.ptr(x, np.float32), a.ptr(y, np.float32), a.ptr(t_rel, np.float32)
        if out is None:
            out = _empty_like(x, n, np.int32)
        po = a.ptr(out, np.int32)
        self._check(lib().ecmd_probe_pixels(self.h, C.byref(sensor), px, py, pt, n, float(tau), float(d),
                                            a.flags, po))
        return out

    def probe_point(self, sensor: Sensor, x, y, t_rel, tau: float, d, want_image: bool = False, polarity=None):
        a = _Args()
        n = int(x.shape[0])
        m = int(d.shape[0])
        px, py, pt = a.ptr(x, np.float32), a.ptr(y, np.float32), a.ptr(t_rel, np.float32)
        pp = a.ptr(polarity, np.int8)
        pd = a.ptr(d, np.float32)
        S = _empty_like(x, m, np.uint64)
        N = _empty_like(x, m, np.int64)
        cells = sensor.width * sensor.height * (1 if polarity is None else 2)
        img = _empty_like(x, m * cells, np.uint32) if want_image else None
        self._check(lib().ecmd_probe_point(self.h, C.byref(sensor), px, py, pt, pp, n, float(tau), pd, m, a.flags,
                                           a.ptr(S, np.uint64), a.ptr(N, np.int64),
                                           a.ptr(img, np.uint32) if want_image else None))
        return (S, N, img) if want_image else (S, N)

    def probe_bound(self, sensor: Sensor, x, y, t_rel, tau: float, d_lo: float, d_hi: float, d_a, d_b,
                    want_image: bool = False, polarity=None):
        a = _Args()
        n = int(x.shape[0])
        m = int(d_a.shape[0])
        px, py, pt = a.ptr(x, np.float32), a.ptr(y, np.float32), a.ptr(t_rel, np.float32)
        pp = a.ptr(polarity, np.int8)
        pa, pb = a.ptr(d_a, np.float32), a.ptr(d_b, np.float32)
        S = _empty_like(x, m, np.uint64)
        N = _empty_like(x, m, np.int64)
        cells = sensor.width * sensor.height * (1 if polarity is None else 2)
        img = _empty_like(x, m * cells, np.uint32) if want_image else None
        self._check(lib().ecmd_probe_bound(self.h, C.byref(sensor), px, py, pt, pp, n, float(tau), float(d_lo),
                                           float(d_hi), pa, pb, m, a.flags, a.ptr(S, np.uint64),
                                           a.ptr(N, np.int64), a.ptr(img, np.uint32) if want_image else None))
        return (S, N, img) if want_image else (S, N)

    def estimate_learned(self, cnn: "Cnn", sensor: Sensor, x, y, t_rel, offsets, tau, d_lo: float, d_hi: float,
                         eps: float, gamma: float = 0.0, max_nodes: int = 0, frontier_batch: int = 0,
                         frontier_capacity: int = 0, exact_bounds: bool = False) -> list:
        """Batched estimation whose incumbents are seeded by the network."""
        a = _Args()
        B = int(tau.shape[0])
        px, py, pt = a.ptr(x, np.float32), a.ptr(y, np.float32), a.ptr(t_rel, np.float32)
        po, ptau = a.ptr(offsets, np.int64), a.ptr(tau, np.float32)
        sp = _search(d_lo, d_hi, eps, gamma, max_nodes, frontier_batch, frontier_capacity, exact_bounds)
        out = (ResultS * max(B, 1))()
        rc = lib().ecmd_estimate_divergence_learned(self.h, cnn.h, C.byref(sensor), px, py, pt, po, ptau, B,
                                                    C.byref(sp), a.flags, out)
        self._check(rc, allow=(EBUDGET, EFRONTIER))
        return [Result.of(out[i]) for i in range(B)]

    def estimate_stream(self, sensor: Sensor, x, y, t, t_start: float, tau: float, K: int, d_lo: float,
                        d_hi: float, eps: float, polarity=None, **kw) -> list:
        """K consecutive windows of length tau from t_start (Sec. 4.4)."""
        a = _Args()
        n = int(x.shape[0])
        ev = EventsS(a.ptr(x, np.float32), a.ptr(y, np.float32), a.ptr(t, np.float64), n,
                     a.ptr(polarity, np.int8))
        sp = _search(d_lo, d_hi, eps, **kw)
        out = (ResultS * max(K, 1))()
        rc = lib().ecmd_estimate_stream(self.h, C.byref(sensor), C.byref(ev), float(t_start), float(tau), int(K),
                                        C.byref(sp), a.flags, out)
        self._check(rc, allow=(EBUDGET, EFRONTIER))
        return [Result.of(out[i]) for i in range(K)]

    def _preproc_out(self, x, offsets):
        n = int(offsets[-1] - offsets[0])
        B = int(offsets.shape[0]) - 1
        return (_empty_like(x, max(n, 1), np.float32), _empty_like(x, max(n, 1), np.float32),
                _empty_like(x, max(n, 1), np.float32), _empty_like(x, B + 1, np.int64))

    def hot_pixel_filter(self, sensor: Sensor, x, y, t_rel, offsets, max_count: int):
        """Drop the events of pixels holding more than max_count events of
        their window (Sec. 6 preprocessing); returns (x, y, t_rel, offsets)."""
        a = _Args()
        B = int(offsets.shape[0]) - 1
        xo, yo, to, oo = self._preproc_out(x, offsets)
        self._check(lib().ecmd_hot_pixel_filter(self.h, C.byref(sensor), a.ptr(x, np.float32), a.ptr(y, np.float32),
                                                a.ptr(t_rel, np.float32), a.ptr(offsets, np.int64), B, int(max_count),
                                                a.flags, a.ptr(xo, np.float32), a.ptr(yo, np.float32),
                                                a.ptr(to, np.float32), a.ptr(oo, np.int64)))
        m = int(oo[-1])
        return xo[:m], yo[:m], to[:m], oo

    def resample(self, in_sensor: Sensor, out_sensor: Sensor, x, y, t_rel, offsets, keep_frac: float, seed: int):
        """Resized and resampled events (Sec. 6); returns (x, y, t_rel, offsets)."""
        a = _Args()
        B = int(offsets.shape[0]) - 1
        xo, yo, to, oo = self._preproc_out(x, offsets)
        self._check(lib().ecmd_resample(self.h, C.byref(in_sensor), C.byref(out_sensor), a.ptr(x, np.float32),
                                        a.ptr(y, np.float32), a.ptr(t_rel, np.float32), a.ptr(offsets, np.int64), B,
                                        float(keep_frac), C.c_uint64(seed), a.flags, a.ptr(xo, np.float32),
                                        a.ptr(yo, np.float32), a.ptr(to, np.float32), a.ptr(oo, np.int64)))
        m = int(oo[-1])
        return xo[:m], yo[:m], to[:m], oo

    def downsample(self, sensor: Sensor, x, y, offsets):
        a = _Args()
        B = int(offsets.shape[0]) - 1
        px, py, po = a.ptr(x, np.float32), a.ptr(y, np.float32), a.ptr(offsets, np.int64)
        out = _empty_like(x, B * GRID * GRID, np.uint16)
        self._check(lib().ecmd_downsample(self.h, C.byref(sensor), px, py, po, B, a.flags, a.ptr(out, np.uint16)))
        return out


class BatchPlan:
    """An asynchronous batched search (``ecmd_plan_*``): ``launch`` only
    enqueues kernels on the context's stream and writes ``ecmd_result``
    records into a caller buffer (see ``result_buffer``), so it can be
    captured into a graph."""

    def __init__(self, ctx: Context, sensor: Sensor, search: SearchS, limits: PlanLimitsS):
        self.ctx = ctx
        h = C.c_void_p()
        rc = lib().ecmd_plan_create(ctx.h, C.byref(sensor), C.byref(search), C.byref(limits), C.byref(h))
        ctx._check(rc)
        self.h = h
        self.limits = {f: getattr(limits, f) for f, _ in PlanLimitsS._fields_ if f != "reserved"}

    def close(self):
        if getattr(self, "h", None):
            lib().ecmd_plan_destroy(self.h)
            self.h = None

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def result_buffer(B: int, device: bool = True):
        """A torch byte buffer for B results: on the GPU, or pinned host memory."""
        import torch

        n = C.sizeof(ResultS) * max(int(B), 1)
        if device:
            return torch.zeros(n, dtype=torch.uint8, device="cuda")
        return torch.zeros(n, dtype=torch.uint8, pin_memory=True)

    def launch(self, x, y, t_rel, offsets, tau, out, d_seeds=None, polarity=None):
        """Enqueue the search of len(tau) windows (torch CUDA tensors); the
        results land in ``out`` when the stream reaches them."""
        a = _Args()
        B = int(tau.shape[0])
        args = [a.ptr(x, np.float32), a.ptr(y, np.float32), a.ptr(t_rel, np.float32),
                a.ptr(polarity, np.int8) if polarity is not None else None, a.ptr(offsets, np.int64),
                a.ptr(tau, np.float32), B, a.ptr(d_seeds, np.float32) if d_seeds is not None else None]
        if not a.device:
            raise TypeError("plan launches take device arrays")
        if out.numel() < C.sizeof(ResultS) * B:
            raise ValueError("result buffer too small")
        rc = lib().ecmd_plan_launch(self.h, *args, C.c_void_p(out.data_ptr()))
        self.ctx._check(rc)

    @staticmethod
    def results(out, B: int) -> list:
        """Decode B results from a result buffer (after the stream reached them)."""
        raw = out.detach().cpu().numpy().tobytes()
        arr = (ResultS * B).from_buffer_copy(raw[:C.sizeof(ResultS) * B])
        return [Result.of(arr[i]) for i in range(B)]


class Cnn:
    """The learned-incumbent network of a context (parameters on the GPU)."""

    def __init__(self, ctx: Context, seed: int = 0):
        h = C.c_void_p()
        ctx._check(lib().ecmd_cnn_create(ctx.h, C.c_uint64(seed), C.byref(h)))
        self.h = h
        self.ctx = ctx

    def close(self):
        if getattr(self, "h", None):
            lib().ecmd_cnn_destroy(self.h)
            self.h = None

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass

    def params(self) -> np.ndarray:
        p = np.empty(CNN_NPARAM, np.float32)
        self.ctx._check(lib().ecmd_cnn_get_params(self.h, p.ctypes.data))
        return p

    def set_params(self, p: np.ndarray):
        p = np.ascontiguousarray(p, np.float32)
        assert p.shape == (CNN_NPARAM,)
        self.ctx._check(lib().ecmd_cnn_set_params(self.h, p.ctypes.data))

    def save(self, path: str):
        """Checkpoint: parameters and Adam state (resumes training exactly)."""
        self.ctx._check(lib().ecmd_cnn_save(self.h, os.fsencode(path)))

    def load(self, path: str):
        self.ctx._check(lib().ecmd_cnn_load(self.h, os.fsencode(path)))

    def forward(self, imgs):
        a = _Args()
        B = int(imgs.shape[0]) if imgs.ndim > 1 else int(imgs.shape[0]) // (GRID * GRID)
        pi = a.ptr(imgs, np.uint16)
        out = _empty_like(imgs, B, np.float32)
        self.ctx._check(lib().ecmd_cnn_forward(self.h, pi, B, a.flags, a.ptr(out, np.float32)))
        return out

    def grads(self, imgs, labels):
        a = _Args()
        B = int(labels.shape[0])
        pi, pl = a.ptr(imgs, np.uint16), a.ptr(labels, np.float32)
        g = np.empty(CNN_NPARAM, np.float32)
        loss = C.c_float()
        self.ctx._check(lib().ecmd_cnn_grads(self.h, pi, pl, B, a.flags, g.ctypes.data, C.byref(loss)))
        return g, float(loss.value)

    def train_step(self, imgs, labels, lr: float) -> float:
        a = _Args()
        B = int(labels.shape[0])
        pi, pl = a.ptr(imgs, np.uint16), a.ptr(labels, np.float32)
        loss = C.c_float()
        self.ctx._check(lib().ecmd_cnn_train_step(self.h, pi, pl, B, float(lr), a.flags, C.byref(loss)))
        return float(loss.value)


def _empty_like(ref, n: int, dtype):
    if _is_torch(ref):
        import torch

        tdt = {np.int32: torch.int32, np.int64: torch.int64, np.uint64: torch.int64, np.uint32: torch.int32,
               np.uint16: torch.int16, np.float32: torch.float32}[dtype]
        return torch.empty(n, dtype=tdt, device=ref.device)
    return np.empty(n, dtype)


def sensor(width: int, height: int, foe: Sequence[float]) -> Sensor:
    return Sensor(int(width), int(height), float(foe[0]), float(foe[1]))
