"""Request serving with continuous batching over resident volumes.

Volumes stay resident on the device with their workspaces and hierarchies;
requests are either a TF edit (rebuild of that volume's hierarchy) or a
render (camera + image size).  The loop admits arrived requests in arrival
order into a batch while the device-memory budget allows (resident volumes
and workspaces, plus the output images of batches still on the GPU), enqueues
the batch -- rebuilds first, then the batch's renders in one
``esk_render_batch`` launch per volume dtype -- and goes on admitting the next batch while the
previous ones execute; a batch's memory is released when its completion
event has fired.  A render admitted after a TF edit of the same volume sees
that edit; a TF edit that arrives after a render of the same volume closes
the batch, so every result equals the one obtained by serving the requests
one at a time in arrival order.

Only marshalling and scheduling live here; all work runs in libesk's kernels.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

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


@dataclass
class _Batch:
    reqs: list
    event: object
    out_bytes: int


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
        nz, ny, nx = vol.shape
        need = workspace_bytes((nx, ny, nz), _dtype_code(vol), brick, max_tf) + vol.numel() * vol.element_size()
        if self.resident + need > self.budget:
            raise MemoryError(f"volume {name} needs {need} B; {self.budget - self.resident} B left in the budget")
        ctx = Context(self.device)
        ctx.set_volume(vol, brick, value_range, max_tf=max_tf)
        if tf is not None:
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
        queue = collections.deque()
        inflight = collections.deque()
        t0 = clock()
        nxt = 0
        out_in_flight = 0
        free = self.budget - self.resident
        while nxt < len(reqs) or queue or inflight:
            now = clock() - t0
            while nxt < len(reqs) and reqs[nxt].arrival <= now:
                queue.append(reqs[nxt])
                nxt += 1
            # retire finished batches (frees their output memory)
            while inflight and inflight[0].event.query():
                b = inflight.popleft()
                t = clock() - t0
                for r in b.reqs:
                    r.done = t
                out_in_flight -= b.out_bytes
            # admit the next batch in arrival order
            batch, rendered, out_bytes = [], set(), 0
            while queue and len(batch) < self.max_batch:
                r = queue[0]
                if r.kind == "rebuild" and r.volume in rendered:
                    break                               # keep arrival-order semantics
                need = r.size[0] * r.size[1] * 16 if r.kind == "render" else 0
                if out_in_flight + out_bytes + need > free:
                    break                               # wait for memory to free up
                queue.popleft()
                r.admitted = now
                if r.kind == "render":
                    rendered.add(r.volume)
                out_bytes += need
                batch.append(r)
            if batch:
                self._enqueue(batch)
                ev = torch.cuda.Event()
                ev.record()
                inflight.append(_Batch(batch, ev, out_bytes))
                out_in_flight += out_bytes
                continue
            if queue and not inflight:
                raise MemoryError(f"request {queue[0].rid} does not fit the device-memory budget")
            if inflight:
                if queue or nxt >= len(reqs):
                    inflight[0].event.synchronize()     # blocked on memory, or draining
                else:
                    time.sleep(min(1e-4, max(0.0, reqs[nxt].arrival - (clock() - t0))))
            elif nxt < len(reqs):
                time.sleep(max(0.0, min(1e-3, reqs[nxt].arrival - (clock() - t0))))
        makespan = clock() - t0
        return self._summary(reqs, makespan)

    def _enqueue(self, batch):
        torch = self.torch
        renders = []
        for r in batch:
            if r.kind == "rebuild":
                self.contexts[r.volume].set_tf(r.tf, build=(self.accel,))
            else:
                W, H = r.size
                r.out = torch.empty((H, W, 4), dtype=torch.float32, device="cuda")
                renders.append(r)
        # one batched launch per volume dtype (a launch serves one dtype)
        groups = collections.OrderedDict()
        for r in renders:
            groups.setdefault(self.contexts[r.volume].dtype_code, []).append(r)
        for code, rs in groups.items():
            ctxs = [self.contexts[r.volume] for r in rs]
            buf = self.args_buffers.get(code)
            render_batch(ctxs, [r.cam for r in rs], [r.size for r in rs], accel=self.accel,
                         step=self.step, ref=self.ref, outs=[r.out for r in rs], args_buffer=buf)
            self.args_buffers[code] = ctxs[0]._keep["batch_args"]

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
