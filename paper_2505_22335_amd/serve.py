"""ctypes binding of the request loop (include/asgs_serve.h) plus the host
helpers that drive it: request specs, arrival traces, latency statistics.

The scheduler, admission, batching, streams and the loss all run natively in
libasgs; this module marshals arguments and summarises results.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import _lib as L
from .pipeline import DeviceAnchors

TRACK, MAP = 0, 1
P = C.c_void_p
PP = C.POINTER(C.c_void_p)


class ServerConfig(C.Structure):
    _fields_ = [("n_streams", C.c_int32), ("max_batch_views", C.c_int32), ("fifo", C.c_int32),
                ("simulate", C.c_int32), ("arena_bytes", C.c_uint64), ("sim_us_per_mpix", C.c_float),
                ("sim_us_fixed", C.c_float)]


class Request(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n_views", C.c_int32), ("cams", C.POINTER(L.Camera)),
                ("target_rgb", PP), ("target_depth", PP), ("target_feat", PP), ("weight", P),
                ("d_pose", P), ("loss", P), ("d_xyz", P), ("d_feat", P), ("d_off", P), ("d_params", P),
                ("out_rgb", PP), ("out_depth", PP), ("arrival", C.c_double)]


class Result(C.Structure):
    _fields_ = [("status", C.c_int32), ("batch_views", C.c_int32), ("stream", C.c_int32),
                ("attempts", C.c_int32), ("arrival", C.c_double), ("start", C.c_double), ("done", C.c_double)]


class Stats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("failed", C.c_int64),
                ("batches", C.c_int64), ("batch_views", C.c_int64), ("reruns", C.c_int64),
                ("arena_bytes", C.c_uint64), ("arena_peak", C.c_uint64), ("max_in_flight", C.c_int32),
                ("reserved", C.c_int32)]


_sigs = {
    "asgs_server_create": (C.c_int, [C.POINTER(ServerConfig), C.POINTER(L.Decoder), P, P, P, P,
                                     C.POINTER(L.RenderOpts), C.POINTER(P)]),
    "asgs_server_clock": (C.c_double, []),
    "asgs_server_submit": (C.c_int, [P, C.POINTER(Request), C.POINTER(C.c_uint64)]),
    "asgs_server_wait": (C.c_int, [P, C.c_uint64, C.POINTER(Result)]),
    "asgs_server_replay": (C.c_int, [P, C.POINTER(Request), C.c_int64, C.POINTER(Result)]),
    "asgs_server_stats": (C.c_int, [P, C.POINTER(Stats)]),
    "asgs_server_destroy": (C.c_int, [P]),
}
for _name, (_res, _args) in _sigs.items():
    _f = getattr(L.lib, _name)
    _f.restype = _res
    _f.argtypes = _args


def _ptrs(ts) -> Optional[C.Array]:
    if ts is None:
        return None
    return (C.c_void_p * len(ts))(*[t.data_ptr() for t in ts])


@dataclass
class RequestSpec:
    """One request: cameras (objects with width, height, fx, fy, cx, cy,
    T_wc), per-view target tensors, output tensors (device, caller-owned)."""
    kind: int
    cams: Sequence
    target_rgb: Sequence[torch.Tensor]
    target_depth: Sequence[torch.Tensor]
    d_pose: torch.Tensor
    target_feat: Optional[Sequence[torch.Tensor]] = None
    weight: Optional[torch.Tensor] = None
    loss: Optional[torch.Tensor] = None
    d_xyz: Optional[torch.Tensor] = None
    d_feat: Optional[torch.Tensor] = None
    d_off: Optional[torch.Tensor] = None
    d_params: Optional[torch.Tensor] = None
    out_rgb: Optional[Sequence[torch.Tensor]] = None
    out_depth: Optional[Sequence[torch.Tensor]] = None
    arrival: float = -1.0
    _keep: list = field(default_factory=list, repr=False)

    def to_c(self) -> Request:
        cams = L.make_cameras(self.cams)
        arrs = [_ptrs(self.target_rgb), _ptrs(self.target_depth), _ptrs(self.target_feat),
                _ptrs(self.out_rgb), _ptrs(self.out_depth)]
        self._keep = [cams] + arrs
        r = Request()
        r.kind, r.n_views = self.kind, len(self.cams)
        r.cams = C.cast(cams, C.POINTER(L.Camera))
        r.target_rgb, r.target_depth, r.target_feat, r.out_rgb, r.out_depth = [
            C.cast(a, PP) if a is not None else None for a in arrs]
        r.weight = L._ptr(self.weight)
        r.d_pose = L._ptr(self.d_pose)
        r.loss = L._ptr(self.loss)
        r.d_xyz, r.d_feat, r.d_off, r.d_params = (L._ptr(self.d_xyz), L._ptr(self.d_feat), L._ptr(self.d_off),
                                                  L._ptr(self.d_params))
        r.arrival = float(self.arrival)
        return r


class Server:
    """A request loop over a resident anchor scene (see asgs_serve.h)."""

    def __init__(self, anchors: Optional[DeviceAnchors], n_anchors: int = 0, k: int = 10, n_feat: int = 16,
                 precision: int = 0, n_streams: int = 2, max_batch_views: int = 16, fifo: bool = False,
                 arena_bytes: int = 32 << 30, simulate: bool = False, sim_us_per_mpix: float = 0.0,
                 sim_us_fixed: float = 0.0, **opt_kw):
        if anchors is not None:
            n_anchors, k, n_feat, l_o, l_s = anchors.A, anchors.k, anchors.n_feat, anchors.l_o, anchors.l_s
        else:
            l_o, l_s = 1.0, 0.02
        self.anchors = anchors
        self.desc = L.make_decoder(n_anchors, k, n_feat, precision, l_o, l_s)
        self.n_params = L.decode_param_count(self.desc)
        self.A, self.k, self.nf = n_anchors, k, n_feat
        self.opts = L.make_opts(n_feat, **opt_kw)
        cfg = ServerConfig(n_streams, max_batch_views, int(fifo), int(simulate), int(arena_bytes),
                           float(sim_us_per_mpix), float(sim_us_fixed))
        h = C.c_void_p()
        ptr = (lambda t: None) if anchors is None else L._ptr
        a = anchors
        if not simulate:
            torch.cuda.synchronize()  # scene tensors written before the server threads read them
        L.check(L.lib.asgs_server_create(C.byref(cfg), C.byref(self.desc), ptr(a and a.xyz), ptr(a and a.feat),
                                         ptr(a and a.off), ptr(a and a.params), C.byref(self.opts), C.byref(h)),
                "asgs_server_create")
        self.h = h
        self.simulate = bool(simulate)

    def _inputs_ready(self):
        # the server's streams do not order against torch's: inputs written
        # by torch must be complete before a request is queued
        if not self.simulate:
            torch.cuda.current_stream().synchronize()

    @staticmethod
    def clock() -> float:
        return L.lib.asgs_server_clock()

    def submit(self, spec: RequestSpec) -> int:
        r = spec.to_c()
        self._inputs_ready()
        t = C.c_uint64()
        L.check(L.lib.asgs_server_submit(self.h, C.byref(r), C.byref(t)), "asgs_server_submit")
        return t.value

    def wait(self, ticket: int) -> Result:
        res = Result()
        L.check(L.lib.asgs_server_wait(self.h, ticket, C.byref(res)), "asgs_server_wait")
        return res

    def replay(self, specs: Sequence[RequestSpec]) -> List[Result]:
        """Submit specs[i] at replay start + specs[i].arrival seconds; wait for all."""
        arr = (Request * len(specs))(*[s.to_c() for s in specs])
        out = (Result * len(specs))()
        self._inputs_ready()
        L.check(L.lib.asgs_server_replay(self.h, arr, len(specs), out), "asgs_server_replay")
        return list(out)

    def stats(self) -> Stats:
        s = Stats()
        L.check(L.lib.asgs_server_stats(self.h, C.byref(s)), "asgs_server_stats")
        return s

    def close(self):
        if self.h:
            L.check(L.lib.asgs_server_destroy(self.h), "asgs_server_destroy")
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def poisson_arrivals(rng: np.random.Generator, rate: float, t_end: float, t0: float = 0.0) -> np.ndarray:
    """Arrival times of a Poisson process of the given rate on [t0, t_end)."""
    out, t = [], t0
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= t_end:
            return np.asarray(out)
        out.append(t)


def latency_summary(results: Sequence[Result], kinds: Sequence[int], t_from: float = 0.0) -> dict:
    """p50/p99/mean latency (ms) per request kind and overall, over requests
    arriving at or after t_from (relative to the first arrival)."""
    arr = np.array([r.arrival for r in results])
    lat = np.array([r.done - r.arrival for r in results]) * 1e3
    ok = np.array([r.status == 0 for r in results])
    kinds = np.asarray(kinds)
    sel = (arr - arr.min() >= t_from) & ok if len(arr) else ok
    out = {}
    for name, m in (("all", sel), ("track", sel & (kinds == TRACK)), ("map", sel & (kinds == MAP))):
        if m.sum() == 0:
            continue
        out[name] = {"n": int(m.sum()), "p50_ms": round(float(np.percentile(lat[m], 50)), 3),
                     "p99_ms": round(float(np.percentile(lat[m], 99)), 3),
                     "mean_ms": round(float(lat[m].mean()), 3)}
    out["failed"] = int((~ok).sum())
    return out
