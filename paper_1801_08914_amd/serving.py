"""Continuous-batching request loop for hybridization solves.

A request is one problem (mesh, order, alpha, beta) with one or more loads
f_1..f_R (implicit time steps).  Requests are admitted, in arrival order with
first fit, as soon as a slot and enough device memory (the plan's buffer
footprint) are free; each admitted request runs on its own HIP stream in its
own host thread, so the work of requests that overlap in time overlaps on the
device.  The factors stay on the device for all loads of a request: load 1
runs setup (matrix and right-hand side), loads 2..R only the right-hand side,
each followed by the Jacobi-PCG solve and the recovery of u.

The numerical path is the library's; results do not depend on what else is
running (deterministic kernels and reductions), which the tests check.
"""
from __future__ import annotations

import collections
import dataclasses
import threading
import time
from concurrent.futures import Future

import numpy as np

from . import Plan


@dataclasses.dataclass
class Request:
    xyz: np.ndarray
    e2v: np.ndarray
    k: int
    alpha: np.ndarray
    beta: np.ndarray
    loads: list            # element-constant loads f_r, each (ne, 3)
    arrival: float = 0.0   # seconds on the server's clock (time.perf_counter() - t0)
    tag: object = None


@dataclasses.dataclass
class Result:
    tag: object
    u: list                # recovered u for every load, (ne, n) host arrays
    iters: list            # PCG iterations per load
    converged: bool
    footprint: int         # device bytes reserved for the request
    elements: int
    arrival: float
    admitted: float
    done: float

    @property
    def latency(self) -> float:
        return self.done - self.arrival


def footprint_bytes(sizes) -> int:
    """Device bytes of a bound plan plus u (the admission measure)."""
    s = sizes
    return int(s.bytes_maps + s.bytes_factor + s.bytes_y + 8 * (s.m + 1) + 4 * s.nnz + 8 * s.nnz + 8 * s.m
               + s.bytes_work + 16 + 2 * 8 * s.m + 8 * s.ne * s.n_local)


class Server:
    """Admit requests by slots and device-memory budget; run them overlapped."""

    def __init__(self, budget_bytes: int, slots: int = 4, rtol: float = 1e-12, maxit: int = 20000,
                 device: str = "cuda:0"):
        import torch
        self.budget = int(budget_bytes)
        self.slots = int(slots)
        self.rtol, self.maxit = rtol, maxit
        self.device = torch.device(device)
        self.t0 = time.perf_counter()
        self._cv = threading.Condition()
        self._waiting: collections.deque = collections.deque()
        self._used = 0
        self._free_slots = self.slots
        self._closing = False
        self._streams = [torch.cuda.Stream(device=self.device) for _ in range(self.slots)]
        self._free_streams = list(range(self.slots))
        self._threads: list[threading.Thread] = []
        self._dispatcher = threading.Thread(target=self._dispatch, daemon=True)
        self._dispatcher.start()

    def now(self) -> float:
        return time.perf_counter() - self.t0

    # ------------------------------------------------------------------ API
    def submit(self, req: Request) -> Future:
        """Plan the request on the host (topology and buffer sizes) and queue
        it; the future resolves to a Result."""
        plan = Plan(req.xyz, req.e2v, req.k)
        need = footprint_bytes(plan.sizes)
        fut: Future = Future()
        if need > self.budget:
            fut.set_exception(MemoryError(f"request needs {need} bytes, budget is {self.budget}"))
            return fut
        with self._cv:
            self._waiting.append((req, plan, need, fut))
            self._cv.notify_all()
        return fut

    def close(self):
        with self._cv:
            self._closing = True
            self._cv.notify_all()
        self._dispatcher.join()
        for t in self._threads:
            t.join()

    # ------------------------------------------------------------- internals
    def _dispatch(self):
        while True:
            with self._cv:
                while True:
                    pick = None
                    if self._free_slots > 0:
                        for i, (_, _, need, _) in enumerate(self._waiting):
                            if self._used + need <= self.budget:
                                pick = i
                                break
                    if pick is not None:
                        break
                    if self._closing and not self._waiting:
                        return
                    self._cv.wait()
                req, plan, need, fut = self._waiting[pick]
                del self._waiting[pick]
                self._used += need
                self._free_slots -= 1
                sid = self._free_streams.pop()
            t = threading.Thread(target=self._run, args=(req, plan, need, fut, sid), daemon=True)
            self._threads.append(t)
            t.start()

    def _release(self, need: int, sid: int):
        with self._cv:
            self._used -= need
            self._free_slots += 1
            self._free_streams.append(sid)
            self._cv.notify_all()

    def _run(self, req: Request, plan: Plan, need: int, fut: Future, sid: int):
        import torch
        admitted = self.now()
        try:
            stream = self._streams[sid]
            with torch.cuda.stream(stream):
                plan.set_stream(stream)
                plan.bind(self.device)
                us, iters, conv = [], [], True
                for r, f in enumerate(req.loads):
                    if r == 0:
                        plan.setup(req.alpha, req.beta, f)
                        # a failed element (non-SPD matrix, det J <= 0) ends
                        # the request here, before its solve
                        rc, det = plan.status()
                        if rc != 0:
                            raise RuntimeError(f"device error {rc} at element {det}")
                    else:
                        plan.rhs(f)
                    lam, info = plan.pcg(self.rtol, self.maxit)
                    u = plan.recover(lam)
                    us.append(u.cpu().numpy())
                    iters.append(info["iters"])
                    conv = conv and info["converged"]
                rc, det = plan.status()
                if rc != 0:
                    raise RuntimeError(f"device error {rc} at element {det}")
                stream.synchronize()
            res = Result(req.tag, us, iters, conv, need, plan.ne, req.arrival, admitted, self.now())
            del plan
            fut.set_result(res)
        except Exception as exc:  # noqa: BLE001 - delivered to the caller
            fut.set_exception(exc)
        finally:
            self._release(need, sid)


def run_stream(server: Server, requests, realtime: bool = True):
    """Submit (arrival_s, Request) pairs, waiting for each arrival time on the
    server's clock when realtime (otherwise all at once), and return the
    results in submission order.  A request's arrival is its submission time."""
    futs = []
    for arrival, req in requests:
        if realtime:
            dt = arrival - server.now()
            if dt > 0:
                time.sleep(dt)
        req.arrival = server.now()
        futs.append(server.submit(req))
    return [f.result() for f in futs]


def latency_stats(results) -> dict:
    lat = np.array([r.latency for r in results])
    el = sum(r.elements * len(r.u) for r in results)
    span = max(r.done for r in results) - min(r.arrival for r in results)
    return {"requests": len(results), "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "mean_s": float(lat.mean()), "req_per_s": len(results) / span, "element_solves_per_s": el / span,
            "span_s": span}
