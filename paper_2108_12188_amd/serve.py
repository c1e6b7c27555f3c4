"""Continuous-batching serving loop for Poisson solves.

Requests (a mesh and a forcing each) arrive over time.  The scheduler admits
them in arrival order while a slot is free and their device-memory
footprint fits in the budget, hands them to the engine, and steps the
engine one round at a time; requests that arrive while others run join at
the next round boundary, and finished ones leave and free their memory.
The GPU engine drives the native continuous-batching server of libsem
(``sem_server_*``): all admitted solves advance together in batched
launches, and each result is bitwise the one the request would get alone.

Host side only: the scheduler holds no arithmetic of the method.  Mesh
preparation for newly admitted requests runs on a worker thread so that it
overlaps the device work of the requests already running.
"""
from __future__ import annotations

import collections
import concurrent.futures as cf
import math
import threading
import time
from dataclasses import dataclass, field

__all__ = ["Request", "Scheduler", "GpuEngine", "summarize"]


@dataclass
class Request:
    tag: int
    arrival: float          # seconds after the start of the run
    n_elem: int
    order: int
    payload: dict = field(default_factory=dict)
    # filled in by the scheduler
    admitted: float = -1.0
    done: float = -1.0
    status: str = "waiting"
    result: dict | None = None


class Scheduler:
    """Admission by slot and memory footprint, FIFO (optionally with
    backfilling of smaller requests behind a blocked head)."""

    def __init__(self, engine, budget_bytes: int, max_slots: int = 64, backfill: bool = False,
                 on_done=None):
        self.engine = engine
        self.on_done = on_done      # called with the number of finished requests
        self.budget = int(budget_bytes)
        self.max_slots = int(max_slots)
        self.backfill = backfill
        self.used = 0
        self.peak_used = 0
        self.active: dict[int, int] = {}
        self.log: list[tuple] = []
        self.finished = 0

    def _try_admit(self, waiting: collections.deque, now: float):
        while waiting and len(self.active) < self.max_slots:
            admitted_one = False
            for k, r in enumerate(waiting):
                fp = self.engine.footprint(r)
                if fp > self.budget:
                    r.status = "rejected"
                    r.done = now
                    del waiting[k]
                    self.log.append(("reject", r.tag, now))
                    admitted_one = True
                    break
                if self.used + fp <= self.budget:
                    del waiting[k]
                    r.status = "running"
                    r.admitted = now
                    self.active[r.tag] = fp
                    self.used += fp
                    self.peak_used = max(self.peak_used, self.used)
                    self.engine.admit(r)
                    self.log.append(("admit", r.tag, now))
                    admitted_one = True
                    break
                if not self.backfill:
                    break
            if not admitted_one:
                break

    def run(self, requests):
        pending = sorted(requests, key=lambda r: (r.arrival, r.tag))
        by_tag = {r.tag: r for r in pending}
        waiting: collections.deque = collections.deque()
        i = 0
        while i < len(pending) or waiting or self.active:
            now = self.engine.now()
            while i < len(pending) and pending[i].arrival <= now:
                waiting.append(pending[i])
                i += 1
            self._try_admit(waiting, now)
            if not self.active:
                if i < len(pending):
                    self.engine.wait_until(pending[i].arrival)
                    continue
                if waiting:          # only possible if the head can never fit
                    r = waiting.popleft()
                    r.status = "rejected"
                    continue
                break
            for tag, res in self.engine.step():
                r = by_tag[tag]
                r.done = self.engine.now()
                r.status = "done" if res.get("converged") else "failed"
                r.result = res
                self.used -= self.active.pop(tag)
                self.engine.release(tag)
                self.log.append(("done", tag, r.done))
                self.finished += 1
                if self.on_done is not None:
                    self.on_done(self.finished)
        return pending


def summarize(requests) -> dict:
    done = [r for r in requests if r.status in ("done", "failed")]
    lat = sorted(r.done - r.arrival for r in done)

    def pct(p):
        if not lat:
            return None
        k = min(len(lat) - 1, max(0, int(math.ceil(p / 100.0 * len(lat))) - 1))
        return lat[k]

    span = (max(r.done for r in done) - min(r.arrival for r in requests)) if done else 0.0
    return {"requests": len(requests), "completed": len(done),
            "converged": sum(1 for r in done if r.status == "done"),
            "rejected": sum(1 for r in requests if r.status == "rejected"),
            "p50_s": pct(50), "p99_s": pct(99), "mean_s": (sum(lat) / len(lat)) if lat else None,
            "solves_per_s": (len(done) / span) if span > 0 else None, "span_s": span}


class GpuEngine:
    """Engine on the native server.  `make_problem(request)` returns
    (vert, glob_id, dirichlet, N, forcing) where forcing(xyz) maps the
    device coordinates [3][n] of the mesh's GLL points to the source f."""

    def __init__(self, make_problem, tol: float = 1e-8, geom: int = 0, inner_tol: float = 0.0,
                 round_iters: int = 16, prep_workers: int = 1, keep_results: bool = False):
        import torch

        from . import MIXED, PRECOMPUTED, Mesh, Server, mesh_footprint
        self._torch = torch
        self._Mesh = Mesh
        self._fp = mesh_footprint
        self._mixed = MIXED
        self.geom = geom
        self.g_fp32 = geom == PRECOMPUTED
        self.server = Server(tol=tol, geom=geom, inner_tol=inner_tol, round_iters=round_iters)
        self.make_problem = make_problem
        self.pool = cf.ThreadPoolExecutor(max_workers=prep_workers)
        self.release_pool = cf.ThreadPoolExecutor(max_workers=1)
        self.preparing: dict[int, cf.Future] = {}
        self.held: dict[int, tuple] = {}
        self.keep_results = keep_results
        self.results: dict[int, object] = {}
        self.peak_measured_bytes = 0
        # host time split: preparation (summed over the worker threads) and
        # the scheduling thread's waits and server rounds
        self.timing = collections.Counter()
        self._lock = threading.Lock()
        self._kept_bytes = 0        # results of released requests kept for the caller
        self._alloc0 = torch.cuda.memory_allocated()
        self.t0 = time.perf_counter()

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def wait_until(self, t: float):
        dt = t - self.now()
        if dt > 0:
            time.sleep(dt)

    # Device bytes per local point a request holds beyond its mesh handle
    # and solver work vectors: its FP64 right-hand side and solution (16),
    # and while it is prepared the point coordinates [3][n] (24), the
    # forcing (8) and at most two temporaries of the forcing expression (16).
    CALLER_BYTES_PER_POINT = 16 + 24 + 8 + 16

    def footprint(self, r: Request) -> int:
        n = r.n_elem * (r.order + 1) ** 3
        return self._fp(r.n_elem, r.order, g_fp32=self.g_fp32, prec=self._mixed) \
            + self.CALLER_BYTES_PER_POINT * n

    def _measure(self):
        """Device bytes held right now by the admitted requests: their mesh
        handles (as the library reports them) plus the tensors this engine
        allocated since it was created."""
        torch = self._torch
        held = sum(m.info()["device_bytes"] for m, _, _ in self.held.values())
        tensors = max(0, torch.cuda.memory_allocated() - self._alloc0 - self._kept_bytes)
        self.peak_measured_bytes = max(self.peak_measured_bytes, held + tensors)

    def _prepare(self, r: Request):
        torch = self._torch
        t0 = time.perf_counter()
        vert, gid, dirichlet, N, forcing = self.make_problem(r)
        t1 = time.perf_counter()
        mesh = self._Mesh(vert, gid, dirichlet, N, g_fp32=self.g_fp32)
        t2 = time.perf_counter()
        f = forcing(mesh.coords())
        b = mesh.rhs(f.contiguous(), prec=self._mixed)
        x = torch.zeros_like(b)
        torch.cuda.current_stream().synchronize()
        t3 = time.perf_counter()
        with self._lock:
            self.timing["make_problem_s"] += t1 - t0
            self.timing["mesh_create_s"] += t2 - t1
            self.timing["rhs_s"] += t3 - t2
        return mesh, b, x

    def admit(self, r: Request):
        self.preparing[r.tag] = self.pool.submit(self._prepare, r)

    def _add_ready(self, block: bool):
        ready = [t for t, f in self.preparing.items() if f.done()]
        if not ready and block and self.preparing:
            t = min(self.preparing)
            self.preparing[t].result()
            ready = [t]
        for t in ready:
            mesh, b, x = self.preparing.pop(t).result()
            self.server.add(mesh, b, x, t)
            self.held[t] = (mesh, b, x)

    def step(self):
        t0 = time.perf_counter()
        self._add_ready(block=not self.held)
        t1 = time.perf_counter()
        if not self.held:
            with self._lock:
                self.timing["wait_prepared_s"] += t1 - t0
            return []
        self._measure()
        done, _ = self.server.step()
        with self._lock:
            self.timing["wait_prepared_s"] += t1 - t0
            self.timing["server_step_s"] += time.perf_counter() - t1
            self.timing["rounds"] += 1
        return done

    def release(self, tag: int):
        mesh, b, x = self.held.pop(tag)
        if self.keep_results:
            self.results[tag] = x
            self._kept_bytes += x.numel() * x.element_size()
        # destroying a mesh synchronises the device and frees its arrays:
        # done on a thread of its own so the scheduling thread goes on
        # feeding the server (the server no longer holds the request)
        self.release_pool.submit(self._destroy, mesh, b)

    def _destroy(self, mesh, b):
        t0 = time.perf_counter()
        mesh.close()
        del b
        with self._lock:
            self.timing["release_s"] += time.perf_counter() - t0

    def close(self):
        self.pool.shutdown(wait=True)
        for t in list(self.held):
            self.release(t)
        self.release_pool.shutdown(wait=True)
        self.server.close()
