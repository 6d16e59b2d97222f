"""Serving loop: continuous batching of orbital-evaluation requests.

Requests come from many Monte Carlo walkers of several resident systems
(each system is one coefficient table kept on the GPU).  A request is one
walker's quasi-simultaneous move block (Sec. IV.A): k positions whose
orbitals, gradients and Laplacians are wanted.  Because every moved electron
is an independent evaluation against its system's table (Eq. (11.12.23.1)),
requests of the same system can be packed into one batched launch and
unpacked afterwards without changing any result.

The scheduler is continuous: whenever a launch slot of a system is free it
packs the waiting requests of that system (FIFO, up to the slot capacity)
into one launch, as long as the HBM budget for in-flight request buffers
allows; launches of different systems, and the two slots of one system, run
on their own streams and overlap on the device.  Requests arriving while
others run are admitted as soon as slots and budget free up.

The scheduler itself is device-agnostic: it drives a backend with
launch / done / fetch calls, so its logic is tested on the CPU with a fake
backend and a fake clock.  :class:`GpuBackend` is the MI355X backend on
libblip (blip_eval_batched captured in hipGraph plans).
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass

import numpy as np

QUEUED, RUNNING, DONE, REJECTED, FAILED, TIMEOUT = (
    "queued", "running", "done", "rejected", "failed", "timeout")


@dataclass
class ServeRequest:
    rid: int
    system: int
    pos: np.ndarray                  # [k, 3] float64, Cartesian bohr
    arrival: float = 0.0             # scheduled arrival time (seconds)
    keep: bool = False               # copy the outputs back on completion
    status: str = QUEUED
    error: str = ""
    t_admit: float = float("nan")
    t_done: float = float("nan")
    result: dict | None = None

    @property
    def npos(self) -> int:
        return int(self.pos.shape[0])

    @property
    def latency(self) -> float:
        return self.t_done - self.arrival


@dataclass
class _Launch:
    system: int
    slot: int
    reqs: list
    handle: object
    nbytes: int


class Server:
    """Continuous-batching scheduler with HBM-budget admission.

    backend must provide:
      nsystems, slots_per_system, capacity(system) -> max positions per launch,
      max_requests(system) -> max requests per launch,
      request_bytes(system, npos) -> device bytes a request holds in flight,
      launch(system, slot, reqs) -> handle   (asynchronous),
      done(handle) -> bool                   (non-blocking poll),
      fetch(system, slot, row0, npos) -> dict of host arrays.
    """

    def __init__(self, backend, budget_bytes: int, timeout_s: float | None = None,
                 clock=None):
        self.b = backend
        self.budget = int(budget_bytes)
        self.timeout = timeout_s
        self.clock = clock or time.perf_counter
        self.queues = [collections.deque() for _ in range(backend.nsystems)]
        self.free_slots = [list(range(backend.slots_per_system)) for _ in range(backend.nsystems)]
        self.running: list[_Launch] = []
        self.inflight = 0
        self.finished: list[ServeRequest] = []
        self.launches = 0
        self.peak_inflight = 0

    # -- arrivals ------------------------------------------------------------

    def offer(self, req: ServeRequest) -> None:
        """A request arrives.  Requests that can never fit are rejected now."""
        if req.system < 0 or req.system >= self.b.nsystems:
            self._finish(req, REJECTED, f"unknown system {req.system}")
            return
        if req.npos < 1:
            self._finish(req, REJECTED, "empty request")
            return
        need = self.b.request_bytes(req.system, req.npos)
        if need > self.budget:
            self._finish(req, REJECTED, f"request needs {need} bytes, budget is {self.budget}")
        elif req.npos > self.b.capacity(req.system):
            self._finish(req, REJECTED,
                         f"request has {req.npos} positions, capacity is {self.b.capacity(req.system)}")
        else:
            req.status = QUEUED
            self.queues[req.system].append(req)

    # -- one scheduling step -----------------------------------------------------

    def pump(self) -> int:
        """Retire finished launches, expire timeouts, admit and launch.
        Returns the number of launches started."""
        now = self.clock()
        self._retire(now)
        if self.timeout is not None:
            self._expire(now)
        return self._admit()

    def _retire(self, now):
        still = []
        for ln in self.running:
            try:
                ok = self.b.done(ln.handle)
            except Exception as e:          # a failed launch fails only its requests
                ok = None
                err = f"{type(e).__name__}: {e}"
            if ok is None:
                t = self.clock()
                for r in ln.reqs:
                    self._finish(r, FAILED, err, t)
                self._release(ln)
            elif ok:
                t = self.clock()
                row = 0
                for r in ln.reqs:
                    if r.keep:
                        try:
                            r.result = self.b.fetch(ln.system, ln.slot, row, r.npos)
                        except Exception as e:
                            self._finish(r, FAILED, f"{type(e).__name__}: {e}", t)
                            row += r.npos
                            continue
                    self._finish(r, DONE, "", t)
                    row += r.npos
                self._release(ln)
            else:
                still.append(ln)
        self.running = still

    def _release(self, ln):
        self.inflight -= ln.nbytes
        self.free_slots[ln.system].append(ln.slot)

    def _expire(self, now):
        for q in self.queues:
            keep = collections.deque()
            while q:
                r = q.popleft()
                if now - r.arrival > self.timeout:
                    self._finish(r, TIMEOUT, f"waited {now - r.arrival:.3f} s", now)
                else:
                    keep.append(r)
            q.extend(keep)

    def _admit(self) -> int:
        started = 0
        # serve the system whose oldest waiting request is oldest first
        order = sorted((q[0].arrival, s) for s, q in enumerate(self.queues) if q)
        for _, s in order:
            q = self.queues[s]
            while q and self.free_slots[s]:
                cap = self.b.capacity(s)
                maxr = self.b.max_requests(s)
                batch, npos, nbytes = [], 0, 0
                while q and len(batch) < maxr:
                    r = q[0]
                    need = self.b.request_bytes(s, r.npos)
                    if npos + r.npos > cap or self.inflight + nbytes + need > self.budget:
                        break
                    batch.append(q.popleft())
                    npos += r.npos
                    nbytes += need
                if not batch:
                    break                  # budget full: wait for completions (FIFO per system)
                slot = self.free_slots[s].pop()
                t = self.clock()
                for r in batch:
                    r.t_admit = t
                    r.status = RUNNING
                try:
                    h = self.b.launch(s, slot, batch)
                except Exception as e:
                    for r in batch:
                        self._finish(r, FAILED, f"{type(e).__name__}: {e}", self.clock())
                    self.free_slots[s].append(slot)
                    continue
                self.inflight += nbytes
                self.peak_inflight = max(self.peak_inflight, self.inflight)
                self.running.append(_Launch(s, slot, batch, h, nbytes))
                self.launches += 1
                started += 1
        return started

    def _finish(self, r, status, err="", t=None):
        r.status = status
        r.error = err
        r.t_done = self.clock() if t is None else t
        self.finished.append(r)

    # -- drivers -----------------------------------------------------------------

    def idle(self) -> bool:
        return not self.running and not any(self.queues)

    def run(self, requests, sleep=None):
        """Open-loop driver: release each request at its scheduled arrival
        time (relative to the start), pump until everything has finished.
        Latency is measured from the scheduled arrival, so a slow scheduler
        shows up in it (no coordinated omission)."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        t0 = self.clock()
        for r in reqs:
            r.arrival = r.arrival + t0
        i = 0
        while i < len(reqs) or not self.idle():
            now = self.clock()
            while i < len(reqs) and reqs[i].arrival <= now:
                self.offer(reqs[i])
                i += 1
            self.pump()
            if sleep is not None and i < len(reqs) and not self.running:
                sleep(min(1e-4, max(0.0, reqs[i].arrival - self.clock())))
        t1 = self.clock()
        for r in reqs:
            r.arrival -= t0
            r.t_done -= t0
            r.t_admit -= t0
        return summarize(reqs, t1 - t0, self)


def summarize(reqs, makespan, server=None, norb=None) -> dict:
    done = [r for r in reqs if r.status == DONE]
    lat = np.array([r.latency for r in done]) if done else np.array([np.nan])
    out = {"requests": len(reqs), "done": len(done),
           "rejected": sum(r.status == REJECTED for r in reqs),
           "failed": sum(r.status == FAILED for r in reqs),
           "timeout": sum(r.status == TIMEOUT for r in reqs),
           "makespan_s": makespan,
           "req_per_s": len(done) / makespan if makespan > 0 else float("nan"),
           "positions": int(sum(r.npos for r in done)),
           "p50_ms": float(np.percentile(lat, 50) * 1e3),
           "p99_ms": float(np.percentile(lat, 99) * 1e3)}
    if done:
        # where the latency goes: waiting for admission (queue), and from
        # admission to the scheduler seeing the completion (staging, the
        # device, and the polling lag)
        wait = np.array([r.t_admit - r.arrival for r in done])
        svc = np.array([r.t_done - r.t_admit for r in done])
        out["queue_wait_p50_ms"] = float(np.percentile(wait, 50) * 1e3)
        out["queue_wait_p99_ms"] = float(np.percentile(wait, 99) * 1e3)
        out["in_service_p50_ms"] = float(np.percentile(svc, 50) * 1e3)
        out["in_service_p99_ms"] = float(np.percentile(svc, 99) * 1e3)
    if server is not None:
        out["launches"] = server.launches
        out["peak_inflight_bytes"] = server.peak_inflight
        host = getattr(server.b, "launch_host_s", None)
        if host is not None and server.launches:
            out["launch_host_us_mean"] = host / server.launches * 1e6
    return out


# ---------------------------------------------------------------------------
# MI355X backend


class GpuBackend:
    """Resident tables on the GPU, two launch slots per system.

    Each slot owns device buffers for up to ``capacity`` positions (positions,
    offsets, val/grad/lap, sort workspace), a pinned host staging buffer, its
    own stream and, for the batched mode, a hipGraph plan of
    blip_eval_batched on those buffers.  A launch packs the requests'
    positions into the staging buffer and makes one library call
    (blip_submit) that copies them host-to-device on the slot's stream,
    evaluates them (or replays the plan) and records the slot's event.

    Launches smaller than ``sort_threshold`` positions skip the spatial sort
    and run one direct blip_eval on the slot's buffers (the host knows the
    packed count); the sort pays only when many positions share rows.  Both
    forms compute every output in the same order, so results are identical.

    batched=False runs one request per launch with ``kernel`` (e.g. the plain
    single-block kernel), the unbatched baseline.
    """

    def __init__(self, tables, capacity: int = 16384, max_requests: int = 512,
                 slots_per_system: int = 2, batched: bool = True, kernel: str = "auto",
                 sort_threshold: int = 4096):
        import torch
        from .blip import Submitter
        self.torch = torch
        self.tables = tables
        self.nsystems = len(tables)
        self.slots_per_system = slots_per_system
        self.batched = batched
        self.kernel = kernel
        self.sort_threshold = sort_threshold
        self._cap = capacity if batched else 1536
        self._maxr = max_requests if batched else 1
        self.sorted_launches = 0      # launches replaying the sorted batched plan
        self.direct_launches = 0      # launches running one blip_eval
        self.launch_host_s = 0.0      # host time spent in launch() (staging + submit)
        dev = torch.device("cuda", torch.cuda.current_device())
        self.slots = []
        for t in tables:
            per = []
            for _ in range(slots_per_system):
                cap = self._cap
                st = torch.cuda.Stream(device=dev)       # default priority
                pos = torch.zeros((cap, 3), dtype=torch.float64, device=dev)
                off = torch.zeros(self._maxr + 1, dtype=torch.int64, device=dev)
                out = t.alloc_outputs(cap, True, dev)
                ws = t.workspace(cap, dev) if batched else None
                hpos = torch.zeros((cap, 3), dtype=torch.float64, pin_memory=True)
                hoff = torch.zeros(self._maxr + 1, dtype=torch.int64, pin_memory=True)
                plan = t.plan(pos, off, out, ws, capacity=cap) if batched else None
                ev = torch.cuda.Event()
                ev.record(st)                    # gives the event its HIP handle
                sub = Submitter(t, hpos, pos, out, st, ev, plan=plan, host_off=hoff,
                                dev_off=off, kernel=kernel if not batched else "auto")
                per.append({"stream": st, "pos": pos, "off": off, "out": out, "ws": ws,
                            "hpos": hpos, "hoff": hoff, "hpos_np": hpos.numpy(),
                            "hoff_np": hoff.numpy(), "plan": plan, "event": ev,
                            "submit": sub})
            self.slots.append(per)
        torch.cuda.synchronize()

    def capacity(self, s):
        return self._cap

    def max_requests(self, s):
        return self._maxr

    def request_bytes(self, s, npos):
        # positions + val/grad/lap rows (float or complex float)
        w = self.tables[s].norb * (2 if self.tables[s].complex else 1)
        return int(npos) * (24 + 5 * 4 * w)

    def launch(self, s, slot, reqs):
        t0 = time.perf_counter()
        sl = self.slots[s][slot]
        hp = sl["hpos_np"]
        # the staging buffers are reused only after this slot's previous
        # launch completed (the scheduler frees a slot on completion)
        # one packing call for the whole launch (a slice assignment per
        # request cost about a microsecond each at saturation)
        counts = [r.npos for r in reqs]
        row = sum(counts)
        if reqs:
            np.concatenate([r.pos for r in reqs], axis=0, out=hp[:row])
        sorted_plan = self.batched and row >= self.sort_threshold
        if sorted_plan:
            ho = sl["hoff_np"]
            ho[0] = 0
            ho[1:len(reqs) + 1] = np.cumsum(counts)
            ho[len(reqs) + 1:] = row
            self.sorted_launches += 1
        else:
            self.direct_launches += 1
        sl["submit"](row, sorted_plan)
        self.launch_host_s += time.perf_counter() - t0
        return (s, slot)

    def done(self, handle):
        s, slot = handle
        return self.slots[s][slot]["event"].query()

    def fetch(self, s, slot, row0, npos):
        sl = self.slots[s][slot]
        sl["event"].synchronize()
        v, g, l = sl["out"]
        return {"val": v[row0:row0 + npos].cpu().numpy(),
                "grad": g[row0:row0 + npos].cpu().numpy(),
                "lap": l[row0:row0 + npos].cpu().numpy()}

    def close(self):
        for per in self.slots:
            for sl in per:
                if sl["plan"] is not None:
                    sl["plan"].free()
        self.slots = []
