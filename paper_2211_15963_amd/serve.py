"""Served stream of simulation requests on one GPU (continuous batching).

The Digital Brain is deployed as a service that clients submit simulations to
(Section "Digital Brain platform" of the main text: users set parameters through
a code interface and the system runs and records the simulation). Here a request is
a seeded network description plus a biological duration. The server:

* admits requests in arrival order while the sum of the admitted requests' exact
  device footprints (dbsim_footprint) stays within an HBM budget and fewer than
  max_active are resident; a request that does not fit waits (no skipping ahead, so
  no request starves);
* builds admitted networks' host tables on a pool of host threads (dbsim_build: no HIP
  call, so construction overlaps with device work), then deploys each from the serving
  thread onto its own HIP stream (dbsim_create_built): every HIP call of the server - and
  torch's - is made by that one thread;
* keeps every admitted network's state resident and advances all of them in slices
  of slice_bins bins, keeping up to two slices queued per stream, so the kernels of
  different requests overlap on the device;
* retires a request when its last slice has completed: reads its results, frees its
  memory and admits the next waiting requests. A request whose build, step or read
  fails retires with the error and frees its memory; the others go on;
* cancels a request at its cancel_at_s (relative to the start) or when cancel(rid) is
  called from another thread: waiting, building or resident, it retires with the error
  "cancelled" and frees what it holds.

Each request's result depends only on its own description (every handle is
independent and bit-deterministic), so a request gives the same bits alone and in
any mix; the tests check exactly that.
"""
from __future__ import annotations

import concurrent.futures as cf
import hashlib
import threading
import time
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np

from .dbsim import Built, DbsimError, Simulator, footprint


@dataclass
class Request:
    rid: int
    spec: object          # netgen NetSpec
    n_steps: int          # Euler steps to run (whole bins for full results)
    arrival_s: float = 0.0
    cancel_at_s: Optional[float] = None  # the client withdraws the request at this time
    # filled by the server
    footprint: int = 0
    t_admit: float = float("nan")
    t_built: float = float("nan")
    t_done: float = float("nan")
    result: Optional[Dict] = None
    error: Optional[str] = None

    @property
    def latency_s(self) -> float:
        return self.t_done - self.arrival_s


def summarize(sim: Simulator, with_state_digest: bool = True, full: bool = False) -> Dict:
    """Result of a finished request: counters, per-bin spike counts (all regions) and a
    digest of the final state (V, J, refractory counters); with full=True also the raster
    (steps, ids) and the final state arrays."""
    st = sim.stats()
    _, cnt = sim.region_signal()
    out = {"steps": st["steps"], "bins": st["bins"], "spikes": st["spikes"], "edge_events": st["edge_events"],
           "bin_spikes": cnt.sum(axis=1).astype(np.int64)}
    state = sim.state() if (with_state_digest or full) else None
    if with_state_digest:
        h = hashlib.sha256()
        for a in state:
            h.update(np.ascontiguousarray(a).tobytes())
        out["state_sha256"] = h.hexdigest()
    if full:
        out["raster"] = sim.spikes()
        out["state"] = state
    return out


@dataclass
class _Active:
    req: Request
    sim: Simulator
    stream: object
    enqueued: int = 0
    inflight: List = field(default_factory=list)  # torch events, oldest first


class Server:
    def __init__(self, hbm_budget: Optional[int] = None, max_active: int = 16, slice_bins: int = 25,
                 build_workers: int = 2, build_threads: Optional[int] = None, device: int = 0,
                 state_digest: bool = True, full_results: bool = False):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible to torch")
        self.torch = torch
        self.device = device
        torch.cuda.set_device(device)
        if hbm_budget is None:
            free, _total = torch.cuda.mem_get_info(device)
            hbm_budget = int(free * 0.85)
        self.hbm_budget = int(hbm_budget)
        self.max_active = int(max_active)
        self.slice_bins = int(slice_bins)
        self.build_workers = int(build_workers)
        if build_threads is None:
            import os
            total = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or (os.cpu_count() or 1)
            build_threads = max(1, total // max(1, self.build_workers))
        self.build_threads = int(build_threads)
        self.state_digest = state_digest
        self.full_results = full_results
        self._lock = threading.Lock()
        self._cancelled: set = set()

    def cancel(self, rid: int) -> None:
        """Withdraws request rid (callable from any thread while run() serves)."""
        with self._lock:
            self._cancelled.add(rid)

    def _is_cancelled(self, r: Request, now: float) -> bool:
        if r.cancel_at_s is not None and now >= r.cancel_at_s:
            return True
        with self._lock:
            return r.rid in self._cancelled

    def _build(self, req: Request) -> Built:
        """Host phase, on a pool thread: validation, plan and tables; no HIP or torch call."""
        bins = -(-req.n_steps // req.spec.steps_per_bin)
        return Built(req.spec, record_regions=True, host_threads=self.build_threads, record_bins=max(4096, bins))

    def _deploy(self, req: Request, built: Built):
        """Device phase, on the serving thread: its own stream, memory from torch, upload."""
        stream = self.torch.cuda.Stream(device=self.device)  # default priority
        sim = Simulator(req.spec, record_regions=True, device=self.device, stream=stream, built=built)
        return sim, stream

    def run(self, requests: List[Request], poll_s: float = 2e-4) -> Dict:
        """Serves the requests on the real clock (arrival_s relative to the start) and
        returns the per-request records and the aggregate statistics."""
        torch = self.torch
        pending = sorted(requests, key=lambda r: r.arrival_s)
        for r in pending:
            bins = -(-r.n_steps // r.spec.steps_per_bin)
            r.footprint = footprint(r.spec, record_regions=True, record_bins=max(4096, bins))
            if r.footprint > self.hbm_budget:
                r.error = f"footprint {r.footprint} B exceeds the HBM budget {self.hbm_budget} B"
        waiting: List[Request] = []
        building: Dict[cf.Future, Request] = {}
        active: List[_Active] = []
        done: List[Request] = []
        in_use = 0
        peak_active = 0
        pool = cf.ThreadPoolExecutor(max_workers=self.build_workers)
        t0 = time.perf_counter()
        i = 0
        try:
            while i < len(pending) or waiting or building or active:
                now = time.perf_counter() - t0
                progressed = False
                while i < len(pending) and pending[i].arrival_s <= now:
                    r = pending[i]
                    i += 1
                    if r.error:
                        r.t_done = now
                        done.append(r)
                    else:
                        waiting.append(r)
                # withdrawn requests that hold nothing yet
                for r in [r for r in waiting if self._is_cancelled(r, now)]:
                    waiting.remove(r)
                    r.error, r.t_done = "cancelled", now
                    done.append(r)
                    progressed = True
                # admission: arrival order, by footprint and slot
                while (waiting and len(active) + len(building) < self.max_active
                       and in_use + waiting[0].footprint <= self.hbm_budget):
                    r = waiting.pop(0)
                    in_use += r.footprint
                    r.t_admit = now
                    building[pool.submit(self._build, r)] = r
                    progressed = True
                # finished builds are deployed (here, on the serving thread) and join the active set
                for fut in [f for f in building if f.done()]:
                    r = building.pop(fut)
                    if self._is_cancelled(r, time.perf_counter() - t0):
                        if fut.exception() is None:
                            fut.result().free()
                        r.error, r.t_done = "cancelled", time.perf_counter() - t0
                        in_use -= r.footprint
                        done.append(r)
                        progressed = True
                        continue
                    try:
                        sim, stream = self._deploy(r, fut.result())
                    except Exception as ex:  # a failed build or deploy retires the request with its error
                        r.error = str(ex)
                        r.t_done = time.perf_counter() - t0
                        in_use -= r.footprint
                        done.append(r)
                        continue
                    r.t_built = time.perf_counter() - t0
                    active.append(_Active(r, sim, stream))
                    progressed = True
                peak_active = max(peak_active, len(active))
                # keep up to two slices queued per resident network
                for a in active:
                    while a.inflight and a.inflight[0].query():
                        a.inflight.pop(0)
                    while a.req.error is None and len(a.inflight) < 2 and a.enqueued < a.req.n_steps:
                        n = min(self.slice_bins * a.sim.S, a.req.n_steps - a.enqueued)
                        try:
                            with torch.cuda.stream(a.stream):
                                a.sim.step(n)
                                ev = torch.cuda.Event()
                                ev.record(a.stream)
                        except DbsimError as ex:
                            a.req.error = str(ex)
                            break
                        a.inflight.append(ev)
                        a.enqueued += n
                        progressed = True
                # retire finished, failed and withdrawn requests (destroy waits for the handle's stream)
                still = []
                now = time.perf_counter() - t0
                for a in active:
                    if a.req.error is None and self._is_cancelled(a.req, now):
                        a.req.error = "cancelled"
                    if a.req.error is not None or (a.enqueued >= a.req.n_steps and not a.inflight):
                        if a.req.error is None:
                            try:
                                a.sim.sync()
                                a.req.result = summarize(a.sim, self.state_digest, self.full_results)
                            except DbsimError as ex:
                                a.req.error = str(ex)
                        a.sim.close()
                        a.req.t_done = time.perf_counter() - t0
                        in_use -= a.req.footprint
                        done.append(a.req)
                        progressed = True
                    else:
                        still.append(a)
                active = still
                if not progressed:
                    time.sleep(poll_s)
        finally:
            pool.shutdown(wait=True)
            # on an exception, free what is still resident or built
            for a in active:
                a.sim.close()
            for fut in building:
                if fut.done() and fut.exception() is None:
                    fut.result().free()
        wall = time.perf_counter() - t0
        ok = [r for r in done if r.error is None]
        lat = np.array([r.latency_s for r in ok]) if ok else np.zeros(1)
        events = sum(r.result["edge_events"] for r in ok)
        return {"requests": done, "wall_s": wall, "completed": len(ok), "failed": len(done) - len(ok),
                "p50_latency_s": float(np.percentile(lat, 50)), "p99_latency_s": float(np.percentile(lat, 99)),
                "events_per_s": events / wall, "peak_active": peak_active,
                "mean_wait_s": float(np.mean([r.t_admit - r.arrival_s for r in ok])) if ok else 0.0,
                "mean_build_s": float(np.mean([r.t_built - r.t_admit for r in ok])) if ok else 0.0}
