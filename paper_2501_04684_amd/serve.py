"""Serving loop: continuous batching of far-zone GMRES solves on one GPU.

Requests (a box geometry, 1..8 right-hand sides) arrive over time. Each one
is planned on a host thread, admitted when a slot and enough device memory
are free (its footprint is known exactly before admission: plan workspace +
Krylov workspace + its two vectors), and then advanced a few Arnoldi steps
at a time on its own HIP stream, so the steps of different requests overlap
on the device. A finished request releases its memory at once and the next
one in arrival order is admitted: requests join and leave at step
boundaries rather than in fixed batches. All device work runs in the
library's kernels; this module only schedules.

Each request's arithmetic depends on nothing but its own inputs (no shared
buffers, no atomics, fixed reduction orders), so a result computed in the
mix is the result computed alone.
"""
from __future__ import annotations

import concurrent.futures as cf
import math
import time
from dataclasses import dataclass, field

import numpy as np

from . import (FarField, Solver, gmres_workspace_bytes, plan_create, plan_destroy,
               workspace_bytes, profile_begin, profile_end)

__all__ = ["Request", "Result", "Server", "auto_shift", "footprint_bytes", "SHIFT_ITERS"]

SHIFT_ITERS = 3  # power-iteration rounds of the automatic shift


@dataclass
class Request:
    """One solve of (sigma I + Z^F) x = b for the geometry ``boxes``."""

    rid: int
    boxes: np.ndarray                 # (n, 3) int32 box coordinates
    b: np.ndarray                     # (nrhs, n * N_u) complex64, host
    arrival: float = 0.0              # seconds after the start of the run
    a: float = 0.25
    k: float = 2.0 * math.pi
    n_d: int = 3
    far_mode: str = "ilist"
    precision: str = "split-bf16"
    tol: float = 1e-4
    restart: int = 30
    max_steps: int = 300
    sigma: complex | None = None      # None: auto_shift of the geometry

    @property
    def nrhs(self) -> int:
        return int(self.b.shape[0])


@dataclass
class Result:
    rid: int
    x: np.ndarray | None
    converged: bool
    steps: int
    restarts: int
    max_rel_res: float
    sigma: complex
    t_arrival: float
    t_admit: float
    t_done: float
    footprint: int
    nrhs: int
    error: str | None = None
    stage_ms: np.ndarray | None = None  # summed stage times of its products (profiling)
    products_timed: int = 0
    setup_products: int = 0             # single-RHS products of the shift estimate
    n_pairs: int = 0                    # far-zone box pairs of its geometry
    translate_flops: float = 0.0        # real flops of one product, one RHS

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrival

    @property
    def products(self) -> int:
        """Far-zone products of the solve (per right-hand side): one per
        step and one per restart."""
        return self.steps + self.restarts


def auto_shift(solver: Solver, iters: int = None, seed: int = 0) -> complex:
    """Set and return sigma = 2 ||Z^F||_2 e^{j pi/4} for the solver's plan, so
    that ||Z^F / sigma|| < 1 and GMRES on sigma I + Z^F contracts the residual
    by about 1/2 per step. ||Z^F||_2 comes from power iteration on Z^H Z run
    on the device (``iters`` rounds of two products, from below)."""
    est = solver.norm_estimate(SHIFT_ITERS if iters is None else iters, seed)
    sigma = complex(2.0 * est * np.exp(0.25j * np.pi))
    solver.set_shift(sigma)
    return sigma


def footprint_bytes(plan, nrhs: int, restart: int) -> int:
    """Device bytes a request holds while active."""
    info_n = _nb_total(plan)
    return (workspace_bytes(plan, nrhs) + gmres_workspace_bytes(plan, nrhs, restart)
            + 2 * nrhs * info_n * 8 + 3 * 256)


def _nb_total(plan) -> int:
    from . import plan_info
    i = plan_info(plan)
    return i["n_boxes"] * i["n_u"]


def _build(req: Request):
    return plan_create(req.boxes, req.a, req.k, req.n_d, req.far_mode, 0.0, req.precision)


@dataclass
class _Active:
    req: Request
    field: FarField
    solver: Solver
    stream: object
    b: object
    x: object
    sigma: complex
    t_admit: float
    footprint: int
    t_arrival: float = 0.0
    draining: bool = False
    done_event: object = None
    status: dict = field(default_factory=dict)


class Server:
    """Continuous-batching GMRES server on one GPU.

    ``hbm_budget``: device bytes the active requests may hold together;
    ``max_active``: concurrent requests (each on its own stream);
    ``steps_per_tick``: Arnoldi steps enqueued for a request each time its
    previous steps have completed; ``profile``: record HIP events around
    the stages of one product in ``profile_every`` of each request.
    """

    def __init__(self, hbm_budget: int, max_active: int = 16, steps_per_tick: int = 2,
                 plan_threads: int = 8, device: str = "cuda", profile: bool = False,
                 profile_every: int = 1):
        import torch
        self.budget = int(hbm_budget)
        self.max_active = int(max_active)
        self.steps_per_tick = int(steps_per_tick)
        self.device = device
        self.pool = cf.ThreadPoolExecutor(max_workers=plan_threads)
        self.streams = [torch.cuda.Stream(device=device) for _ in range(self.max_active)]
        self.log = []          # (time, n_active, bytes in use) after each admission/release
        self.peak_active = 0
        self.profile = bool(profile)  # HIP events around the stages of products
        self.profile_every = max(1, int(profile_every))

    def close(self):
        self.pool.shutdown(wait=True)

    def _admit(self, req: Request, plan, t0: float, stream, fp: int) -> _Active:
        # Memory comes from torch's current (default) stream and is used on
        # the request's stream only after the request's work there is done,
        # so freed blocks are safe for any later request.
        import torch
        ff = FarField.from_plan(plan, max_nrhs=req.nrhs, device=self.device, stream=stream)
        solver = Solver(ff, 0.0 if req.sigma is None else req.sigma, nrhs=req.nrhs,
                        restart=req.restart, tol=req.tol, max_steps=req.max_steps,
                        stream=stream)
        sigma = req.sigma if req.sigma is not None else auto_shift(solver)
        if self.profile:
            profile_begin(ff.plan, self._max_products(req), self.profile_every)
        b = torch.from_numpy(np.ascontiguousarray(req.b)).to(self.device)
        x = torch.empty_like(b)
        stream.wait_stream(torch.cuda.current_stream())
        solver.start(b, x)
        return _Active(req, ff, solver, stream, b, x, sigma, time.perf_counter() - t0, fp)

    @staticmethod
    def _max_products(req: Request) -> int:
        return req.max_steps + req.max_steps // req.restart + 2

    def run(self, requests, realtime: bool = True) -> list[Result]:
        """Serve ``requests`` (arrival times in seconds from now when
        ``realtime``, else all at once) and return their results in rid
        order."""
        import torch
        pending = sorted(requests, key=lambda r: (r.arrival, r.rid))
        building = []                 # (req, future, t_arrival)
        ready = []                    # (req, plan, t_arrival), arrival order
        active: list[_Active] = []
        free_streams = list(self.streams)
        results = {}
        in_use = 0
        t0 = time.perf_counter()
        n_total = len(pending)
        while len(results) < n_total:
            now = time.perf_counter() - t0
            progressed = False
            while pending and (not realtime or pending[0].arrival <= now):
                r = pending.pop(0)
                t_arr = r.arrival if realtime else 0.0
                building.append((r, self.pool.submit(_build, r), t_arr))
                progressed = True
            still = []
            for r, fut, t_arr in building:
                if fut.done():
                    try:
                        ready.append((r, fut.result(), t_arr))
                    except Exception as e:  # invalid geometry: reported, not served
                        results[r.rid] = Result(r.rid, None, False, 0, 0, math.inf, 0j,
                                                t_arr, now, now, 0, r.nrhs, str(e))
                    progressed = True
                else:
                    still.append((r, fut, t_arr))
            building = still
            ready.sort(key=lambda e: (e[2], e[0].rid))
            # admission: arrival order, while a slot and the memory are free
            while ready and free_streams:
                r, plan, t_arr = ready[0]
                fp = footprint_bytes(plan, r.nrhs, r.restart)
                if fp > self.budget:
                    ready.pop(0)
                    plan_destroy(plan)
                    results[r.rid] = Result(r.rid, None, False, 0, 0, math.inf, 0j, t_arr,
                                            now, now, fp, r.nrhs,
                                            f"needs {fp} bytes, budget {self.budget}")
                    progressed = True
                    continue
                if in_use + fp > self.budget:
                    break
                ready.pop(0)
                a = self._admit(r, plan, t0, free_streams.pop(), fp)
                a.t_arrival = t_arr
                in_use += fp
                active.append(a)
                self.peak_active = max(self.peak_active, len(active))
                self.log.append((time.perf_counter() - t0, len(active), in_use))
                progressed = True
            # progress of the active requests
            keep = []
            for a in active:
                if a.draining:
                    if a.done_event.query():
                        t_done = time.perf_counter() - t0
                        st = a.status
                        out = Result(
                            a.req.rid, a.x.cpu().numpy(), bool(st["converged"]), st["steps"],
                            st["restarts"], float(st["max_rel_res"]), a.sigma, a.t_arrival,
                            a.t_admit, t_done, a.footprint, a.req.nrhs)
                        out.n_pairs = a.field.info["n_pairs"]
                        out.setup_products = 0 if a.req.sigma is not None else 2 * SHIFT_ITERS
                        out.translate_flops = a.field.info["translate_flops"]
                        if self.profile:
                            stage, calls = profile_end(a.field.plan, self._max_products(a.req))
                            out.stage_ms, out.products_timed = stage, len(calls)
                        results[a.req.rid] = out
                        a.solver.close()
                        a.field.close()
                        in_use -= a.footprint
                        free_streams.append(a.stream)
                        self.log.append((t_done, len(active) - 1, in_use))
                        progressed = True
                        continue
                    keep.append(a)
                    continue
                st = a.solver.poll(wait=False)
                if not st["ready"]:
                    keep.append(a)
                    continue
                progressed = True
                if st["done"]:
                    a.status = st
                    a.solver.finish()
                    ev = torch.cuda.Event()
                    ev.record(a.stream)
                    a.done_event = ev
                    a.draining = True
                else:
                    for _ in range(self.steps_per_tick):
                        a.solver.step()
                keep.append(a)
            active = keep
            if not progressed:
                time.sleep(0.0002)
        return [results[k] for k in sorted(results)]
