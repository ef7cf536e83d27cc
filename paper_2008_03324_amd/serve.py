"""Continuous-batching request loop over resident Fisher Information Fields.

Several fields stay resident in HBM.  Requests arrive over time, each for one
field: a planner batch (poses -> trace / lambda_min / log-det) or an optimizer
batch (poses -> metrics and their gradients w.r.t. translation and rotation).

The loop admits a waiting request as soon as an in-flight slot is free and its
device buffers fit the HBM budget; admitted requests for the same field and
kind are packed into one launch, launches go round-robin over several HIP
streams so work of different batches overlaps on the device, and each launch
replays a hipGraph captured once per (stream, field, kind, padded size).  A
request completes when the event recorded after its batch has fired; its
latency is completion minus arrival.

Every step of the computation runs in libfif's kernels; this module only moves
requests, buffers and events.  Results are bitwise independent of the mix: a
query's arithmetic depends only on its own pose and the field.
"""
from __future__ import annotations

import dataclasses
import gc
import time
from collections import deque

import torch

import ctypes

from . import (FP64, LMIN, LOGDET, TRACE, CField, CServeConfig, CServeRequest, Field, _check,
               lib, query, query_grad)

METRICS = TRACE | LMIN | LOGDET


class AdmissionError(RuntimeError):
    """A request can never be admitted (it alone exceeds the HBM budget)."""


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float          # seconds since the stream started
    field: int
    kind: str               # "plan" or "opt"
    t: torch.Tensor         # [m, 3] device
    q: torch.Tensor         # [m, 4] device
    # "opt": dL/dout of every pose for trace, lambda_min, log-det (a zero
    # weight leaves that metric out of the gradient)
    weights: tuple = (1.0, 1.0, 1.0)
    # filled by the server
    out: torch.Tensor | None = None      # [m, 3] float64
    grad_t: torch.Tensor | None = None   # [m, 3]
    grad_phi: torch.Tensor | None = None
    admitted: float = float("nan")
    done: float = float("nan")
    status: str = "waiting"

    @property
    def m(self) -> int:
        return int(self.t.shape[0])

    def bytes_needed(self) -> int:
        per = 24 + (48 if self.kind == "opt" else 0) + (24 if self.kind == "opt" else 0)
        return self.m * per


def size_class(m: int, smallest: int = 256) -> int:
    c = smallest
    while c < m:
        c *= 2
    return c


def _fill_weights(up: torch.Tensor, reqs: list[Request]):
    """Each request's metric weights into its rows of the batch's upstream
    buffer, by fills with scalar arguments (no host-to-device copy); runs of
    requests with equal weights share one fill per metric."""
    off = 0
    i = 0
    while i < len(reqs):
        j, n = i, 0
        while j < len(reqs) and reqs[j].weights == reqs[i].weights:
            n += reqs[j].m
            j += 1
        for c, w in enumerate(reqs[i].weights):
            up[off:off + n, c].fill_(float(w))
        off += n
        i = j


class _Lane:
    """One stream with its static buffers and captured graphs."""

    def __init__(self, server: "Server", idx: int):
        self.server = server
        self.idx = idx
        self.stream = torch.cuda.Stream()
        self.graphs = {}
        self.bufs = {}
        self.busy_until = None  # event of the last batch

    def buffers(self, fid: int, kind: str, cap: int):
        key = (fid, kind, cap)
        b = self.bufs.get(key)
        if b is None:
            f = self.server.fields[fid]
            dt = f.pose_dtype
            dev = f.buffer.device
            b = {"t": torch.zeros((cap, 3), dtype=dt, device=dev),
                 "q": torch.zeros((cap, 4), dtype=dt, device=dev),
                 "out": torch.zeros((cap, 3), dtype=torch.float64, device=dev)}
            b["q"][:, 0] = 1.0
            if kind == "opt":
                b["up"] = torch.ones((cap, 3), dtype=torch.float64, device=dev)
                b["gt"] = torch.zeros((cap, 3), dtype=dt, device=dev)
                b["gphi"] = torch.zeros((cap, 3), dtype=dt, device=dev)
            self.bufs[key] = b
        return b

    def launch(self, fid: int, kind: str, cap: int, use_graph: bool):
        f = self.server.fields[fid]
        b = self.buffers(fid, kind, cap)

        def body():
            if kind == "plan":
                query(f, b["t"], b["q"], METRICS, out=b["out"])
            else:
                gt, gphi, out = query_grad(f, b["t"], b["q"], METRICS, b["up"], want_out=True)
                b["gt"].copy_(gt)
                b["gphi"].copy_(gphi)
                b["out"].copy_(out)

        if not use_graph:
            body()
            return
        key = (fid, kind, cap)
        g = self.graphs.get(key)
        if g is None:
            # warm up on this stream, then capture
            body()
            torch.cuda.current_stream().synchronize()
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=self.stream):
                body()
            self.graphs[key] = g
        g.replay()


class Server:
    """Continuous batching over resident fields with HBM-budget admission."""

    def __init__(self, fields: list[Field], n_streams: int = 4, max_inflight: int = 32,
                 hbm_budget: int = 4 << 30, max_batch: int = 65536, use_graphs: bool = True,
                 co_batch: bool = True):
        self.fields = fields
        self.lanes = [_Lane(self, i) for i in range(n_streams)]
        self.max_inflight = max_inflight
        self.hbm_budget = hbm_budget
        self.max_batch = max_batch
        self.use_graphs = use_graphs
        self.co_batch = co_batch
        self.reserved = 0
        self.inflight = []  # (event, [requests], lane)
        self.next_lane = 0

    def warmup(self, caps=(256, 512, 1024, 2048, 4096, 8192, 16384, 32768, 65536)):
        """Allocate the static buffers and capture the graphs of every (stream,
        field, kind, size class) ahead of time, so no capture lands inside the
        timed loop."""
        if not self.use_graphs:
            return
        for lane in self.lanes:
            for fid in range(len(self.fields)):
                for kind in ("plan", "opt"):
                    for cap in caps:
                        if cap > size_class(self.max_batch):
                            continue
                        with torch.cuda.stream(lane.stream):
                            lane.launch(fid, kind, cap, True)
        torch.cuda.synchronize()

    # ----------------------------------------------------------- admission
    def _admit(self, req: Request, now: float) -> bool:
        need = req.bytes_needed()
        if need > self.hbm_budget:
            raise AdmissionError(f"request {req.rid} needs {need} B, budget {self.hbm_budget} B")
        n_in = sum(len(r) for _, r, _ in self.inflight)
        if n_in >= self.max_inflight or self.reserved + need > self.hbm_budget:
            return False
        self.reserved += need
        req.admitted = now
        req.status = "admitted"
        return True

    def _retire(self, now_fn):
        keep = []
        for ev, reqs, lane in self.inflight:
            if ev.query():
                t_done = now_fn()
                for r in reqs:
                    r.done = t_done
                    r.status = "done"
                    self.reserved -= r.bytes_needed()
            else:
                keep.append((ev, reqs, lane))
        self.inflight = keep

    # ----------------------------------------------------------- batching
    def _launch(self, reqs: list[Request]):
        """One batch: a fixed number of launches whatever the number of requests
        (one concatenation per input into the static buffers, the kernel or its
        graph, one copy-out per output; requests receive views of it)."""
        fid, kind = reqs[0].field, reqs[0].kind
        m = sum(r.m for r in reqs)
        lane = self.lanes[self.next_lane]
        self.next_lane = (self.next_lane + 1) % len(self.lanes)
        cap = size_class(m)
        with torch.cuda.stream(lane.stream):
            b = lane.buffers(fid, kind, cap)
            if len(reqs) == 1:
                b["t"][:m].copy_(reqs[0].t)
                b["q"][:m].copy_(reqs[0].q)
            else:
                torch.cat([r.t for r in reqs], out=b["t"][:m])
                torch.cat([r.q for r in reqs], out=b["q"][:m])
            if kind == "opt":
                _fill_weights(b["up"], reqs)
            lane.launch(fid, kind, cap, self.use_graphs)
            out = b["out"][:m].clone()
            if kind == "opt":
                gt = b["gt"][:m].clone()
                gphi = b["gphi"][:m].clone()
            off = 0
            for r in reqs:
                r.out = out[off:off + r.m]
                if kind == "opt":
                    r.grad_t = gt[off:off + r.m]
                    r.grad_phi = gphi[off:off + r.m]
                off += r.m
            ev = torch.cuda.Event()
            ev.record(lane.stream)
        self.inflight.append((ev, reqs, lane))

    def _form_batches(self, admitted: deque):
        groups = {}
        while admitted:
            r = admitted.popleft()
            key = (r.field, r.kind)
            if not self.co_batch:
                self._launch([r])
                continue
            g = groups.setdefault(key, [])
            if g and sum(x.m for x in g) + r.m > self.max_batch:
                self._launch(g)
                groups[key] = g = []
            g.append(r)
        for g in groups.values():
            if g:
                self._launch(g)

    # ----------------------------------------------------------- driver
    def run(self, requests: list[Request], realtime: bool = True, idle_sleep: float = 0.0):
        """Serve the requests in arrival order.  With realtime, a request is not
        seen before its arrival time (wall clock from the start of the run).
        Python's cyclic garbage collector is paused for the duration of the loop
        (its full collections stall the loop for tens of milliseconds)."""
        gc_was_enabled = gc.isenabled()
        gc.collect()
        gc.disable()
        try:
            return self._run(requests, realtime, idle_sleep)
        finally:
            if gc_was_enabled:
                gc.enable()

    def _run(self, requests, realtime, idle_sleep):
        pending = deque(sorted(requests, key=lambda r: r.arrival))
        waiting: deque = deque()
        t0 = time.perf_counter()
        now = lambda: time.perf_counter() - t0  # noqa: E731
        while pending or waiting or self.inflight:
            tn = now()
            while pending and (not realtime or pending[0].arrival <= tn):
                waiting.append(pending.popleft())
            self._retire(now)
            admitted = deque()
            while waiting:
                if self._admit(waiting[0], tn):
                    admitted.append(waiting.popleft())
                else:
                    break
            if admitted:
                self._form_batches(admitted)
            elif idle_sleep:
                time.sleep(idle_sleep)
        torch.cuda.synchronize()
        return now()


class NativeServer:
    """The same loop in libfif (fif_serve_run): admission, packing of requests
    of one field and kind into a launch (one gather kernel, the query or query
    + gradient kernels, one scatter kernel), round-robin over HIP streams and
    completion by events all run in C++ on the calling thread; Python only
    marshals the request list before and reads the times after."""

    def __init__(self, fields: list[Field], n_streams: int = 4, max_inflight: int = 32,
                 hbm_budget: int = 4 << 30, max_batch: int = 65536, co_batch: bool = True):
        self.fields = fields
        self.cfg = CServeConfig(n_streams, max_inflight, hbm_budget, max_batch, int(co_batch), 1)
        nbytes = int(lib().fif_serve_workspace_bytes(ctypes.byref(self.cfg)))
        if nbytes == 0:
            raise ValueError("invalid serving configuration")
        dev = fields[0].buffer.device
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        self.cfields = (CField * len(fields))(*[f.cstruct for f in fields])

    def run(self, requests: list[Request], realtime: bool = True) -> float:
        """Serve the requests; fills out / grad_t / grad_phi, admitted, done and
        status of each; returns the run's length in seconds."""
        n = len(requests)
        arr = (CServeRequest * n)()
        for i, r in enumerate(requests):
            f = self.fields[r.field]
            dt = f.pose_dtype
            if r.t.dtype != dt or r.q.dtype != dt or not (r.t.is_contiguous() and r.q.is_contiguous()):
                raise TypeError(f"request {r.rid}: t and q must be contiguous {dt}")
            r.out = torch.empty((r.m, 3), dtype=torch.float64, device=r.t.device)
            opt = r.kind == "opt"
            if opt:
                r.grad_t = torch.empty((r.m, 3), dtype=dt, device=r.t.device)
                r.grad_phi = torch.empty((r.m, 3), dtype=dt, device=r.t.device)
            arr[i] = CServeRequest(r.arrival, r.field, 1 if opt else 0, r.m, r.t.data_ptr(),
                                   r.q.data_ptr(), r.out.data_ptr(),
                                   r.grad_t.data_ptr() if opt else None,
                                   r.grad_phi.data_ptr() if opt else None,
                                   (ctypes.c_double * 3)(*map(float, r.weights)), 0.0, 0.0)
        self.cfg.realtime = int(realtime)
        elapsed = ctypes.c_double(0.0)
        # the loop creates its streams on the current device: the fields' one
        with torch.cuda.device(self.workspace.device):
            torch.cuda.synchronize()  # request inputs and outputs allocated and ready
            _check(lib().fif_serve_run(self.cfields, len(self.fields), arr, n,
                                       ctypes.byref(self.cfg),
                                       ctypes.c_void_p(self.workspace.data_ptr()),
                                       self.workspace.numel(), ctypes.byref(elapsed)),
                   "fif_serve_run")
        for i, r in enumerate(requests):
            r.admitted, r.done, r.status = arr[i].admitted, arr[i].done, "done"
        return elapsed.value


def latency_stats(requests: list[Request]) -> dict:
    lat = torch.tensor([r.done - r.arrival for r in requests], dtype=torch.float64)
    if lat.numel() == 0:
        return {"n": 0}
    q = torch.quantile(lat, torch.tensor([0.5, 0.99], dtype=torch.float64))
    return {"n": int(lat.numel()), "p50_ms": float(q[0]) * 1e3, "p99_ms": float(q[1]) * 1e3,
            "mean_ms": float(lat.mean()) * 1e3, "max_ms": float(lat.max()) * 1e3}
