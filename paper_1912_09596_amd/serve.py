"""Request serving with continuous batching over resident volumes.

Volumes stay resident on the device with their workspaces and hierarchies,
each on a stream of its own; requests are either a TF edit (rebuild of that
volume's hierarchy) or a render (camera + image size).  The loop admits
arrived requests in arrival order into a batch while the device-memory
budget allows (resident volumes and workspaces, plus the output images of
requests still on the GPU) and enqueues the batch: TF edits on their
volumes' streams, then the renders -- a volume's lone render on its own
stream, several renders of one volume dtype in one ``esk_render_batch``
launch ordered after every involved volume's stream.  Work on different
volumes therefore overlaps on the device (a TF edit of one volume runs
beside another volume's render), and the loop goes on admitting while
earlier batches execute.  A completion thread waits on each request's event
and time-stamps it, which also returns its output memory to the budget.

A render admitted after a TF edit of the same volume sees that edit; a TF
edit that arrives after a render of the same volume closes the batch, and a
volume's stream waits for any batched launch that read its hierarchy, so
every result equals the one obtained by serving the requests one at a time
in arrival order.

Only marshalling and scheduling live here; all work runs in libesk's kernels.
"""
from __future__ import annotations

import collections
import queue as _queue
import threading
import time
from dataclasses import dataclass

from . import Context, render_batch, workspace_bytes, _dtype_code


@dataclass
class Request:
    rid: int
    volume: str
    kind: str                 # "rebuild" or "render"
    arrival: float            # seconds from the start of the run
    tf: object = None         # [N, 4] float32 device tensor (rebuild)
    cam: dict = None          # camera basis (render)
    size: tuple = (0, 0)      # (W, H) (render)
    admitted: float = None
    done: float = None
    out: object = None        # [H, W, 4] float32 device tensor (render)


class Server:
    def __init__(self, hbm_budget_bytes: int, max_batch: int = 64, accel: str = "lbvh", step: float = 0.5,
                 ref: float = 1.0, device: int = 0):
        import torch
        self.torch = torch
        self.budget = int(hbm_budget_bytes)
        self.max_batch = max_batch
        self.accel = accel
        self.step = step
        self.ref = ref
        self.device = device
        self.contexts = {}
        self.resident = 0
        self.args_buffers = {}

    # -- resident volumes ------------------------------------------------------
    def add_volume(self, name: str, vol, brick: int, value_range=(0.0, 1.0), tf=None, max_tf: int = 256):
        torch = self.torch
        nz, ny, nx = vol.shape
        need = workspace_bytes((nx, ny, nz), _dtype_code(vol), brick, max_tf) + vol.numel() * vol.element_size()
        if self.resident + need > self.budget:
            raise MemoryError(f"volume {name} needs {need} B; {self.budget - self.resident} B left in the budget")
        # the volume was written on the current stream; its own stream (default
        # priority) starts after that
        stream = torch.cuda.Stream(self.device)
        stream.wait_stream(torch.cuda.current_stream(self.device))
        vol.record_stream(stream)
        ctx = Context(self.device, stream=stream)
        ctx.set_volume(vol, brick, value_range, max_tf=max_tf)
        if tf is not None:
            tf.record_stream(stream)
            ctx.set_tf(tf, build=(self.accel,))
        self.contexts[name] = ctx
        self.resident += need
        return ctx

    # -- the loop ---------------------------------------------------------------
    def run(self, requests, clock=time.perf_counter):
        """Serves `requests` (arrival times in seconds from now) and returns
        summary statistics; each request gets .done and (renders) .out."""
        torch = self.torch
        reqs = sorted(requests, key=lambda r: (r.arrival, r.rid))
        pending = collections.deque()
        lock = threading.Lock()
        state = {"out_in_flight": 0, "in_flight": 0}
        waits = _queue.Queue()
        # every stream used below starts after what the caller queued
        for ctx in self.contexts.values():
            ctx.stream.wait_stream(torch.cuda.current_stream(self.device))
        t0 = clock()

        def completions():
            while True:
                item = waits.get()
                if item is None:
                    return
                req, ev, nbytes = item
                ev.synchronize()
                t = clock() - t0
                req.done = t
                with lock:
                    state["out_in_flight"] -= nbytes
                    state["in_flight"] -= 1

        waiter = threading.Thread(target=completions, daemon=True)
        waiter.start()
        free = self.budget - self.resident
        nxt = 0
        try:
            while nxt < len(reqs) or pending:
                now = clock() - t0
                while nxt < len(reqs) and reqs[nxt].arrival <= now:
                    pending.append(reqs[nxt])
                    nxt += 1
                # admit the next batch in arrival order
                batch, rendered, out_bytes = [], set(), 0
                with lock:
                    in_flight_bytes = state["out_in_flight"]
                    busy = state["in_flight"]
                while pending and len(batch) < self.max_batch:
                    r = pending[0]
                    if r.kind == "rebuild" and r.volume in rendered:
                        break                               # keep arrival-order semantics
                    need = r.size[0] * r.size[1] * 16 if r.kind == "render" else 0
                    if in_flight_bytes + out_bytes + need > free:
                        break                               # wait for memory to free up
                    pending.popleft()
                    r.admitted = now
                    if r.kind == "render":
                        rendered.add(r.volume)
                    out_bytes += need
                    batch.append(r)
                if batch:
                    with lock:
                        state["out_in_flight"] += out_bytes
                        state["in_flight"] += len(batch)
                    for item in self._enqueue(batch):
                        waits.put(item)
                    continue
                # every wait below releases the interpreter lock, so the
                # completion thread stamps a request as soon as it is done
                if pending:
                    if busy == 0:
                        raise MemoryError(f"request {pending[0].rid} does not fit the device-memory budget")
                    time.sleep(2e-5)                        # blocked on memory
                elif nxt < len(reqs):
                    # until the next arrival: sleep while it is far, then poll
                    wait = reqs[nxt].arrival - (clock() - t0)
                    time.sleep(wait - 2e-4 if wait > 3e-4 else 0)
        finally:
            waits.put(None)
            waiter.join()
        makespan = clock() - t0
        return self._summary(reqs, makespan)

    def _enqueue(self, batch):
        """Enqueues a batch; returns (request, completion event, output bytes)
        for every request."""
        torch = self.torch
        done = []
        renders = []
        for r in batch:
            ctx = self.contexts[r.volume]
            if r.kind == "rebuild":
                r.tf.record_stream(ctx.stream)
                ctx.set_tf(r.tf, build=(self.accel,))
                ev = torch.cuda.Event()
                ev.record(ctx.stream)
                done.append((r, ev, 0))
            else:
                W, H = r.size
                r.out = torch.empty((H, W, 4), dtype=torch.float32, device=f"cuda:{self.device}")
                renders.append(r)
        # one launch per volume dtype (a launch serves one dtype); a lone
        # render goes straight to its volume's stream
        groups = collections.OrderedDict()
        for r in renders:
            groups.setdefault(self.contexts[r.volume].dtype_code, []).append(r)
        for code, rs in groups.items():
            ctxs = [self.contexts[r.volume] for r in rs]
            if len(rs) == 1:
                r, ctx = rs[0], ctxs[0]
                r.out.record_stream(ctx.stream)
                ctx.render(r.cam, r.size[0], r.size[1], accel=self.accel, step=self.step, ref=self.ref,
                           out=r.out)
                ev = torch.cuda.Event()
                ev.record(ctx.stream)
                done.append((r, ev, r.size[0] * r.size[1] * 16))
                continue
            launch = ctxs[0].stream
            seen = {id(launch)}
            for ctx in ctxs[1:]:
                if id(ctx.stream) not in seen:
                    seen.add(id(ctx.stream))
                    launch.wait_stream(ctx.stream)
            with torch.cuda.stream(launch):
                buf = self.args_buffers.get(code)
                for r in rs:
                    r.out.record_stream(launch)
                render_batch(ctxs, [r.cam for r in rs], [r.size for r in rs], accel=self.accel,
                             step=self.step, ref=self.ref, outs=[r.out for r in rs], args_buffer=buf)
                self.args_buffers[code] = ctxs[0]._keep["batch_args"]
            ev = torch.cuda.Event()
            ev.record(launch)
            # later work on these volumes (a TF edit) waits for the launch
            for ctx in ctxs[1:]:
                if ctx.stream is not launch:
                    ctx.stream.wait_event(ev)
            for r in rs:
                done.append((r, ev, r.size[0] * r.size[1] * 16))
        return done

    @staticmethod
    def _summary(reqs, makespan):
        lat = sorted((r.done - r.arrival) * 1e3 for r in reqs)
        rl = sorted((r.done - r.arrival) * 1e3 for r in reqs if r.kind == "render")

        def pct(xs, q):
            if not xs:
                return None
            return xs[min(len(xs) - 1, int(round(q / 100.0 * (len(xs) - 1))))]

        rays = sum(r.size[0] * r.size[1] for r in reqs if r.kind == "render")
        return {"requests": len(reqs), "renders": len(rl), "makespan_s": makespan,
                "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99),
                "render_p50_ms": pct(rl, 50), "render_p99_ms": pct(rl, 99),
                "mrays_per_s": rays / makespan / 1e6 if makespan > 0 else None}
