"""Continuous-batching request loop over the batched C ABI.

Requests (one solve each: initial data, time step count) arrive over time.
The loop admits queued requests in arrival order while their device memory
fits the HBM budget, keeps every admitted run's state resident on the
device, and advances all resident runs together: each iteration launches up
to a chunk of steps of one batch (gr_batch_*) on a compute stream, then --
while the device works -- admits and initialises newly arrived requests on
the default stream.  A run leaves the batch right after its own last step
(gr_batch_update rewrites the batch's argument block in place, ordered on
the compute stream, with no host synchronisation), so a short request never
shortens the chunk of the others; newly admitted runs join at the next
iteration.  A run's result does not depend on the other runs in the batch
(the kernels compute every cell of a run with the same arithmetic), so the
result of a request is the same alone and in the mix.

Latency of a request = completion time - arrival time on the host clock
that also releases the arrivals; the completion time is that of the request's
last step on the device (an event after it, placed on the host clock through
an event recorded and waited for at the start).
"""
from __future__ import annotations

import collections
import time

import numpy as np

from . import grmhd


def run_bytes(grid) -> int:
    """device bytes of one run: q (8), faces (3), prims (5), metric (2 if
    used) field blocks plus the workspace"""
    fs = grmhd.gr_field_stride(grid)
    nf = 8 + 3 + 5 + (2 if grid.metric else 0)
    return nf * fs * 8 + grmhd.gr_workspace_bytes(grid)


class _Slot:
    __slots__ = ("req", "run", "dt", "left", "bytes", "admit")

    def __init__(self, req, run, dt, left, nbytes, admit):
        self.req, self.run, self.dt, self.left, self.bytes, self.admit = req, run, dt, left, nbytes, admit


class Server:
    """hbm_budget: bytes of device memory the resident runs may hold.
    chunk: steps per iteration (a run that finishes inside it leaves the
    batch after its own last step).
    keep: copy each finished run's primitives, faces and conserved
    variables to the host (for checks)."""

    def __init__(self, hbm_budget, device="cuda:0", chunk=4, tune_cache=None, keep=False, max_runs=1024):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.budget = int(hbm_budget)
        self.chunk = int(chunk)
        self.tune_cache = tune_cache
        self.keep = keep
        self.max_runs = max_runs
        self.compute = torch.cuda.Stream(self.device)
        self.init_stream = torch.cuda.current_stream(self.device)

    def serve(self, requests, payload, clock=time.perf_counter):
        """requests: dicts with 'rid', 'arrival' (s from the start), 'steps';
        payload(req) -> workloads.Setup (the request's initial data).
        Returns the list of per-request records and a summary."""
        torch = self.torch
        pending = collections.deque(sorted(requests, key=lambda r: r["arrival"]))
        queue = collections.deque()
        active = []
        used = 0
        batch = None
        dirty = False
        records = []
        peak = 0
        iters = 0
        updates = 0
        t0 = clock()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev0.record(self.compute)
        ev0.synchronize()
        t_ev0 = clock() - t0

        def admit(now):
            nonlocal used, dirty, peak
            while pending and pending[0]["arrival"] <= now:
                queue.append(pending.popleft())
            while queue and len(active) < self.max_runs:
                req = queue[0]
                setup = payload(req)
                nb = run_bytes(grmhd.grid_of(setup))
                if nb > self.budget:
                    raise ValueError("request %s needs %d bytes, more than the whole budget" % (req["rid"], nb))
                if used + nb > self.budget:
                    break
                queue.popleft()
                run = grmhd.Run(setup, device=self.device, stream=self.init_stream)
                dt = run.dt()
                slot = _Slot(req, run, dt, int(req["steps"]), nb, clock() - t0)
                used += nb
                peak = max(peak, used)
                if slot.left == 0:
                    finish(slot, clock() - t0)
                    used -= nb
                    continue
                active.append(slot)
                dirty = True

        def finish(s, t_done):
            rec = dict(rid=s.req["rid"], arrival=s.req["arrival"], admit=s.admit, done=t_done,
                       latency=t_done - s.req["arrival"], steps=int(s.req["steps"]),
                       cells=int(s.run.setup.ncells), fails=None)
            if self.keep:
                rec["prims"] = s.run.prims()
                rec["faces"] = s.run.faces()
                rec["cons"] = s.run.cons()
                rec["fails"] = s.run.fail_count()
            records.append(rec)

        def set_members(slots):
            nonlocal batch, updates
            runs, dts = [s.run for s in slots], [s.dt for s in slots]
            if batch is None:
                self.compute.wait_stream(self.init_stream)  # new runs are initialised on the default stream
                batch = grmhd.Batch(runs, dts, tune_cache=self.tune_cache, stream=self.compute)
            else:
                batch.update(runs, dts)
                updates += 1

        while pending or queue or active:
            admit(clock() - t0)
            if not active:
                if pending:
                    time.sleep(max(0.0, min(pending[0]["arrival"] - (clock() - t0), 0.01)))
                continue
            if dirty:
                self.compute.wait_stream(self.init_stream)
                set_members(active)
                dirty = False
            stepping = list(active)
            finished = []
            for _ in range(min(self.chunk, max(s.left for s in stepping))):
                batch.step()
                for s in stepping:
                    s.left -= 1
                    s.run.t += s.dt
                done_now = [s for s in stepping if s.left == 0]
                if done_now:
                    ev = torch.cuda.Event(enable_timing=True)
                    ev.record(self.compute)
                    finished += [(s, ev) for s in done_now]
                    stepping = [s for s in stepping if s.left > 0]
                    if not stepping:
                        break
                    set_members(stepping)
            end_ev = torch.cuda.Event()
            end_ev.record(self.compute)
            iters += 1
            # host work overlapping the chunk: arrivals and admissions
            admit(clock() - t0)
            end_ev.synchronize()
            gone = set()
            for s, ev in finished:
                finish(s, t_ev0 + ev0.elapsed_time(ev) * 1e-3)
                used -= s.bytes
                gone.add(id(s))
            active = [s for s in active if id(s) not in gone]
            # the batch now holds `stepping`; runs admitted during the chunk
            # (dirty) join at the next iteration
        if batch is not None:
            batch.close()
        makespan = clock() - t0
        lat = np.array([r["latency"] for r in records])
        zc = float(sum(r["cells"] * r["steps"] for r in records))
        arr = [r["arrival"] for r in requests]
        span = max(arr) - min(arr) if len(arr) > 1 else 0.0
        summary = dict(requests=len(records), makespan_s=makespan, zone_cycles=zc,
                       served_zone_cycles_per_s=zc / makespan if makespan > 0 else 0.0,
                       offered_zone_cycles_per_s=zc / span if span > 0 else None,
                       p50_latency_s=float(np.percentile(lat, 50)) if len(lat) else None,
                       p99_latency_s=float(np.percentile(lat, 99)) if len(lat) else None,
                       iterations=iters, batch_updates=updates, peak_resident_bytes=peak,
                       hbm_budget_bytes=self.budget)
        return records, summary
