"""Continuous batching of Crank-Nicolson simulations on one GPU.

Requests arrive over time, each a domain (level set on an n^dim grid), a number
of steps and dt.  The server admits a waiting request when its estimated device
footprint fits the memory budget and a batch slot is free.  A builder thread
builds the admitted request's hierarchy and state, and prepares it for dt, on a
stream of its own while the GPU keeps working on the resident simulations.

The resident simulations advance together at V-cycle granularity
(``lsmg_batch_advance``): each tick gives every member the next piece of its own
step (a step start, a V-cycle, a Newton update, a new linearisation), so a
member whose step converges quickly goes on to its next step while another is
still iterating.  Between ticks, finished builds join and finished simulations
leave; a simulation in the middle of a step keeps its progress when the batch
is rebuilt around it.

Every member's result is bitwise what it would be alone.  The numerics are all
in the HIP library; this module only schedules.
"""
import collections
import queue
import threading
import time

import numpy as np
import torch

from . import lsmg


class Request:
    """One simulation: level set `phi` (n^dim, x fastest) on [lo, hi]^dim, `steps`
    Crank-Nicolson steps of size dt from s = s0, c = c0, boundary value sb."""

    def __init__(self, rid, arrival, dim, n, steps, dt, phi, lo=-1.0, hi=1.0, s0=0.0, c0=1.0, sb=1.0):
        self.id, self.arrival, self.dim, self.n = rid, arrival, dim, n
        self.steps, self.dt, self.phi, self.lo, self.hi = steps, dt, phi, lo, hi
        self.s0, self.c0, self.sb = s0, c0, sb


class _Member:
    def __init__(self, req, H, st, hb, sbytes, t_admit, t_ready):
        self.req, self.H, self.st = req, H, st
        self.bytes = hb + sbytes
        self.t_admit, self.t_ready = t_admit, t_ready
        self.done = 0
        self.cycles = 0
        self.newton = 0
        self.status = lsmg.OK
        self.lat = []
        self.unknowns = 2 * H.level_info(0)["na"]


class Server:
    """params: lsmg parameters shared by every simulation (coarsest_n, precision, ...);
    budget_bytes: device memory the resident simulations may hold (default 80 % of
    the free memory); max_members: batch slots; keep_states: True to return every
    finished simulation's final state, or a set of request ids."""

    def __init__(self, params, budget_bytes=None, max_members=64, autotune=False, keep_states=False,
                 max_ticks=8):
        self.params = params
        if budget_bytes is None:
            free, _ = torch.cuda.mem_get_info()
            budget_bytes = int(0.8 * free)
        self.budget = budget_bytes
        self.max_members = max_members
        self.autotune = autotune
        self.keep_states = keep_states
        self.max_ticks = max_ticks

    def _build(self, req, stream):
        with torch.cuda.stream(stream):
            phi = torch.from_numpy(np.ascontiguousarray(req.phi, dtype=np.float64)).cuda()
            H = lsmg.Hierarchy(phi, req.dim, req.n, req.lo, req.hi, params=self.params, stream=stream)
            st = lsmg.State(H)
            nn = req.n ** req.dim
            s = torch.full((nn,), req.s0, dtype=torch.float64, device="cuda")
            c = torch.full((nn,), req.c0, dtype=torch.float64, device="cuda")
            st.set_grid(s, c)
            H.set_dt(req.dt)
        stream.synchronize()
        return H, st

    def run(self, requests, log=None):
        """Serve `requests` (arrival times in seconds from now); returns a report dict."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        pending = collections.deque(reqs)
        waiting = collections.deque()
        built = queue.Queue()
        todo = queue.Queue()
        bstream = torch.cuda.Stream()
        main = torch.cuda.current_stream()
        errors = []

        def builder():
            while True:
                item = todo.get()
                if item is None:
                    return
                req, t_admit = item
                try:
                    H, st = self._build(req, bstream)
                    hb, sbytes = H.memory_bytes()
                    built.put((req, H, st, hb, sbytes, t_admit, time.perf_counter() - t0))
                except Exception as e:  # reported after the run
                    errors.append((req.id, repr(e)))
                    built.put((req, None, None, 0, 0, t_admit, time.perf_counter() - t0))

        resident = []
        finished = []
        reserved = 0          # estimated bytes of admitted requests not yet built
        used = 0              # bytes held by resident members
        in_build = 0
        steps_log = []        # (t, members, ms, ticks) per advance call
        batch = None
        dirty = False
        t0 = time.perf_counter()
        th = threading.Thread(target=builder, daemon=True)
        th.start()
        try:
            while pending or waiting or in_build or resident:
                now = time.perf_counter() - t0
                while pending and pending[0].arrival <= now:
                    waiting.append(pending.popleft())
                # admission, first come first served, by estimated footprint
                while waiting and len(resident) + in_build < self.max_members:
                    r = waiting[0]
                    est = sum(lsmg.estimate_bytes(r.dim, r.n, self.params, r.lo, r.hi))
                    if used + reserved + est > self.budget and (resident or in_build):
                        break
                    waiting.popleft()
                    reserved += est
                    in_build += 1
                    r._est = est
                    todo.put((r, now))
                # finished builds join at this step boundary
                while True:
                    try:
                        req, H, st, hb, sbytes, t_admit, t_ready = built.get_nowait()
                    except queue.Empty:
                        break
                    in_build -= 1
                    reserved -= req._est
                    if H is None:
                        finished.append(dict(id=req.id, status="build failed"))
                        continue
                    m = _Member(req, H, st, hb, sbytes, t_admit, t_ready)
                    m.est = req._est
                    used += m.bytes
                    resident.append(m)
                    dirty = True
                if not resident:
                    if in_build:
                        time.sleep(0.0005)
                    elif pending:
                        time.sleep(max(0.0, min(0.01, pending[0].arrival - (time.perf_counter() - t0))))
                    continue
                if dirty:
                    batch = lsmg.Batch([m.H for m in resident], stream=main, autotune=self.autotune)
                    dirty = False
                dts = {m.req.dt for m in resident}
                if len(dts) != 1:
                    raise ValueError("resident simulations must share dt")
                ts = time.perf_counter()
                ended, ticks = batch.advance([m.st for m in resident], dts.pop(),
                                             [m.req.steps - m.done for m in resident],
                                             sb_const=[m.req.sb for m in resident], max_ticks=self.max_ticks)
                ms = (time.perf_counter() - ts) * 1e3
                steps_log.append((ts - t0, len(resident), ms, ticks))
                leave = set()
                for k, s, stt, step_ms in ended:
                    m = resident[k]
                    m.lat.append(step_ms)
                    m.cycles += stt["vcycles"]
                    m.newton += stt["newton_iters"]
                    if s == lsmg.OK:
                        m.done += 1
                    else:
                        m.status = s
                    if m.done >= m.req.steps or s != lsmg.OK:
                        leave.add(k)
                keep = []
                for k, m in enumerate(resident):
                    if k not in leave:
                        keep.append(m)
                        continue
                    t_end = time.perf_counter() - t0
                    rec = dict(id=m.req.id, n=m.req.n, dim=m.req.dim, steps=m.done, status=m.status,
                               arrival=m.req.arrival, admitted=m.t_admit, ready=m.t_ready, finished=t_end,
                               unknowns=m.unknowns, cycles=m.cycles, newton=m.newton, bytes=m.bytes,
                               est_bytes=m.est, lat_ms=m.lat)
                    if self.keep_states is True or (self.keep_states and m.req.id in self.keep_states):
                        rec["state"] = m.st.get().cpu().numpy()
                    finished.append(rec)
                    used -= m.bytes
                    m.st.close()
                    m.H.close()
                    dirty = True
                resident = keep
                if dirty:
                    batch = None
                if log:
                    log(f"t={ts - t0:7.3f}s {ticks} ticks over {steps_log[-1][1]} members {ms:7.2f} ms, "
                        f"{len(ended)} steps ended, resident {len(resident)} waiting {len(waiting)} "
                        f"building {in_build}")
        finally:
            todo.put(None)
            th.join()
        t_end = time.perf_counter() - t0
        lat = np.concatenate([np.asarray(f["lat_ms"]) for f in finished if "lat_ms" in f]) \
            if finished else np.zeros(0)
        work = sum(f["unknowns"] * f["cycles"] for f in finished if "unknowns" in f)
        first = min(r.arrival for r in reqs) if reqs else 0.0
        return dict(
            requests=len(reqs), completed=sum(1 for f in finished if f.get("status") == lsmg.OK),
            errors=errors, makespan_s=t_end - first, unknowns_cycles=work,
            throughput=work / max(t_end - first, 1e-9),
            solution_throughput=sum(f["unknowns"] * f["steps"] for f in finished if "unknowns" in f)
            / max(t_end - first, 1e-9),
            p50_step_ms=float(np.percentile(lat, 50)) if lat.size else None,
            p99_step_ms=float(np.percentile(lat, 99)) if lat.size else None,
            busy_s=sum(s[2] for s in steps_log) * 1e-3,
            busy_throughput=work / max(sum(s[2] for s in steps_log) * 1e-3, 1e-9),
            advance_calls=len(steps_log),
            ticks=sum(s[3] for s in steps_log),
            mean_members=float(np.mean([s[1] for s in steps_log])) if steps_log else 0.0,
            max_members=max((s[1] for s in steps_log), default=0),
            queue_wait_s=float(np.mean([f["admitted"] - f["arrival"] for f in finished if "admitted" in f]))
            if finished else 0.0,
            finished=finished,
        )
