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

Krylov lane (krylov_m > 0): a simulation whose first step needed more than
krylov_cycles V-cycles (slow ghost modes) leaves the batch after that step and
runs its remaining steps alone, with flexible GMRES(krylov_m) preconditioned by
one V-cycle (lsmg_params.krylov_m), from a worker thread on the stream it was
built on, while the batch goes on.  The rule depends on the simulation alone,
so its result is still bitwise that of running it alone under the same rule.
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
        self.lane = "batch"
        self.stream = None
        self.unknowns = 2 * H.level_info(0)["na"]


class Server:
    """params: lsmg parameters shared by every simulation (coarsest_n, precision, ...);
    budget_bytes: device memory the resident simulations may hold (default 80 % of
    the free memory); max_members: batch slots; keep_states: True to return every
    finished simulation's final state, or a set of request ids; krylov_m, krylov_cycles:
    the Krylov lane (off for krylov_m = 0)."""

    def __init__(self, params, budget_bytes=None, max_members=64, autotune=False, keep_states=False,
                 max_ticks=8, krylov_m=0, krylov_cycles=60):
        self.params = params
        if budget_bytes is None:
            free, _ = torch.cuda.mem_get_info()
            budget_bytes = int(0.8 * free)
        self.budget = budget_bytes
        self.max_members = max_members
        self.autotune = autotune
        self.keep_states = keep_states
        self.max_ticks = max_ticks
        self.krylov_m = krylov_m
        self.krylov_cycles = krylov_cycles

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
                # with the Krylov lane, each simulation gets a stream of its own, on which
                # it may later run alone
                stream = torch.cuda.Stream() if self.krylov_m > 0 else bstream
                try:
                    H, st = self._build(req, stream)
                    hb, sbytes = H.memory_bytes()
                    built.put((req, H, st, hb, sbytes, t_admit, time.perf_counter() - t0, stream))
                except Exception as e:  # reported after the run
                    errors.append((req.id, repr(e)))
                    built.put((req, None, None, 0, 0, t_admit, time.perf_counter() - t0, stream))

        lane_in = queue.Queue()    # members moving to the Krylov lane (None: stop)
        lane_out = queue.Queue()   # members whose last lane step ended

        def lane():
            active = []
            while True:
                if not active:
                    m = lane_in.get()
                    if m is None:
                        return
                    active.append(m)
                while True:
                    try:
                        m = lane_in.get_nowait()
                    except queue.Empty:
                        break
                    if m is None:
                        lane_in.put(None)
                        break
                    active.append(m)
                for m in list(active):
                    ts = time.perf_counter()
                    try:
                        rc, stt = m.st.step(m.req.dt, sb_const=m.req.sb, check=False)
                    except Exception as e:  # reported after the run
                        errors.append((m.req.id, repr(e)))
                        rc, stt = lsmg.EHIP, dict(vcycles=0, newton_iters=0)
                    m.lat.append((time.perf_counter() - ts) * 1e3)
                    m.cycles += stt["vcycles"]
                    m.newton += stt["newton_iters"]
                    if rc == lsmg.OK:
                        m.done += 1
                    else:
                        m.status = rc
                    if m.done >= m.req.steps or rc != lsmg.OK:
                        active.remove(m)
                        lane_out.put(m)

        resident = []
        in_lane = 0           # members in the Krylov lane
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
        tl = threading.Thread(target=lane, daemon=True)
        if self.krylov_m > 0:
            tl.start()

        def finish(m):
            t_end = time.perf_counter() - t0
            rec = dict(id=m.req.id, n=m.req.n, dim=m.req.dim, steps=m.done, status=m.status,
                       arrival=m.req.arrival, admitted=m.t_admit, ready=m.t_ready, finished=t_end,
                       unknowns=m.unknowns, cycles=m.cycles, newton=m.newton, bytes=m.bytes,
                       est_bytes=m.est, lat_ms=m.lat, lane=m.lane)
            if self.keep_states is True or (self.keep_states and m.req.id in self.keep_states):
                rec["state"] = m.st.get().cpu().numpy()
            finished.append(rec)
            m.st.close()
            m.H.close()
            return m.bytes

        try:
            while pending or waiting or in_build or resident or in_lane:
                now = time.perf_counter() - t0
                while pending and pending[0].arrival <= now:
                    waiting.append(pending.popleft())
                # admission, first come first served, by estimated footprint
                while waiting and len(resident) + in_lane + in_build < self.max_members:
                    r = waiting[0]
                    est = sum(lsmg.estimate_bytes(r.dim, r.n, self.params, r.lo, r.hi))
                    if used + reserved + est > self.budget and (resident or in_build or in_lane):
                        break
                    waiting.popleft()
                    reserved += est
                    in_build += 1
                    r._est = est
                    todo.put((r, now))
                # finished builds join at this step boundary
                while True:
                    try:
                        req, H, st, hb, sbytes, t_admit, t_ready, stream = built.get_nowait()
                    except queue.Empty:
                        break
                    in_build -= 1
                    reserved -= req._est
                    if H is None:
                        finished.append(dict(id=req.id, status="build failed"))
                        continue
                    m = _Member(req, H, st, hb, sbytes, t_admit, t_ready)
                    m.est = req._est
                    m.stream = stream
                    used += m.bytes
                    resident.append(m)
                    dirty = True
                # members whose lane steps ended
                while True:
                    try:
                        m = lane_out.get_nowait()
                    except queue.Empty:
                        break
                    in_lane -= 1
                    used -= finish(m)
                if not resident:
                    if in_build or in_lane:
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
                # with the lane, a member in its first step is stopped at the end of it, so
                # that the rule below sees that step before any other starts
                left = [1 if self.krylov_m > 0 and m.done == 0 else m.req.steps - m.done for m in resident]
                ended, ticks = batch.advance([m.st for m in resident], dts.pop(), left,
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
                    elif self.krylov_m > 0 and m.done == 1 and stt["vcycles"] > self.krylov_cycles:
                        m.lane = "krylov"
                        leave.add(k)
                keep = []
                for k, m in enumerate(resident):
                    if k not in leave:
                        keep.append(m)
                        continue
                    dirty = True
                    if m.lane == "krylov" and m.done < m.req.steps and m.status == lsmg.OK:
                        p = type(self.params).from_buffer_copy(self.params)
                        p.krylov_m = self.krylov_m
                        m.H.set_params(p)
                        in_lane += 1
                        lane_in.put(m)
                        continue
                    used -= finish(m)
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
            if self.krylov_m > 0:
                lane_in.put(None)
                tl.join()
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
            krylov_lane=[f["id"] for f in finished if f.get("lane") == "krylov"],
            finished=finished,
        )
