"""Rebuild + render captured into one HIP graph.

For launch-bound requests (small volumes, small images) the host work per
request -- argument checks, a dozen kernel launches -- can exceed the device
time.  A context created on a dedicated stream can have one "set TF and
rebuild, then render" sequence recorded into a graph (through
torch.cuda.CUDAGraph, which drives HIP stream capture) and replayed: every
replay reads whatever the captured TF buffer holds at that moment and writes
the captured output image.

Only structures whose rebuild needs no host round trip can be captured: the
macrocell grid and the LBVH (the k-d build reads its level count back).
The camera, image size and structure are fixed at capture time.
"""
from __future__ import annotations

from . import Context


class RebuildRenderGraph:
    def __init__(self, vol, brick, tf_entries, cam, size, accel="lbvh", value_range=(0.0, 1.0), device=0):
        import torch
        if accel not in ("grid", "lbvh"):
            raise ValueError("only grid and LBVH rebuilds can be captured (the k-d build synchronises)")
        self.torch = torch
        self.stream = torch.cuda.Stream(device=device)
        self.ctx = Context(device, stream=self.stream)
        W, H = size
        self.tf = torch.zeros((tf_entries, 4), dtype=torch.float32, device=vol.device)
        self.out = torch.empty((H, W, 4), dtype=torch.float32, device=vol.device)
        with torch.cuda.stream(self.stream):
            self.ctx.set_volume(vol, brick, value_range, max_tf=max(256, tf_entries))
            # one eager pass so every kernel has been loaded before capture
            self.ctx.set_tf(self.tf, build=(accel,))
            self.ctx.render(cam, W, H, accel=accel, out=self.out)
        self.stream.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        # relaxed: the library's launchers query and set kernel attributes
        # (no stream work) while the capture is open
        with torch.cuda.graph(self.graph, stream=self.stream, capture_error_mode="relaxed"):
            self.ctx.set_tf(self.tf, build=(accel,))
            self.ctx.render(cam, W, H, accel=accel, out=self.out)

    def replay(self, tf):
        """Copies `tf` into the captured TF buffer and replays the rebuild and
        the render on the graph's stream; returns the output image (valid
        once the stream has reached this point)."""
        torch = self.torch
        with torch.cuda.stream(self.stream):
            self.tf.copy_(tf)
            self.graph.replay()
        return self.out

    def close(self):
        self.stream.synchronize()
        self.graph.reset()
        self.ctx.close()


class BatchRebuildRenderGraph:
    """Many requests -- each a volume with its own TF, camera and image size --
    rebuilt (one batched launch chain) and rendered (one batched launch),
    captured once into a graph on a dedicated stream and replayed with the
    TFs refilled.  The TFs live in one [n, N, 4] buffer, so a replay is one
    copy and one graph launch whatever the number of requests.  A replay
    re-reads the argument uploads that the capture recorded from the first
    context's staging; that context makes no other batched call."""

    def __init__(self, vols, bricks, tf_entries, cams, sizes, accel="lbvh", value_range=(0.0, 1.0), device=0):
        import torch
        from . import rebuild_batch, render_batch
        if accel not in ("grid", "lbvh"):
            raise ValueError("only grid and LBVH rebuilds can be captured (the k-d build synchronises)")
        n = len(vols)
        if not (len(bricks) == n and len(cams) == n and len(sizes) == n):
            raise ValueError("vols, bricks, cams and sizes must have one entry per request")
        self.torch = torch
        self.stream = torch.cuda.Stream(device=device)
        self.ctxs = [Context(device, stream=self.stream) for _ in range(n)]
        dev = vols[0].device
        self.tf_all = torch.zeros((n, tf_entries, 4), dtype=torch.float32, device=dev)
        tfs = list(self.tf_all.unbind(0))
        self.outs = [torch.empty((h, w, 4), dtype=torch.float32, device=dev) for (w, h) in sizes]
        self.stream.wait_stream(torch.cuda.current_stream(device))
        build = (accel,)
        with torch.cuda.stream(self.stream):
            for c, v, b in zip(self.ctxs, vols, bricks):
                c.set_volume(v, b, value_range, max_tf=max(256, tf_entries))
            # one eager pass: loads every kernel and sizes the staging buffers
            rargs = rebuild_batch(self.ctxs, tfs, build=build)
            render_batch(self.ctxs, cams, sizes, accel=accel, outs=self.outs)
            bargs = self.ctxs[0]._keep["batch_args"]
        self.stream.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        # relaxed: the library's launchers query and set kernel attributes
        # (no stream work) while the capture is open
        with torch.cuda.graph(self.graph, stream=self.stream, capture_error_mode="relaxed"):
            rebuild_batch(self.ctxs, tfs, build=build, args_buffer=rargs)
            render_batch(self.ctxs, cams, sizes, accel=accel, outs=self.outs, args_buffer=bargs)
        self._keep = (rargs, bargs, vols)

    def replay(self, tf_stack):
        """Copies the [n, N, 4] TFs into the captured buffer and replays the
        rebuilds and the render on the graph's stream; returns the output
        images (valid once the stream has reached this point)."""
        torch = self.torch
        with torch.cuda.stream(self.stream):
            self.tf_all.copy_(tf_stack)
            self.graph.replay()
        return self.outs

    def close(self):
        self.stream.synchronize()
        self.graph.reset()
        for c in self.ctxs:
            c.close()
