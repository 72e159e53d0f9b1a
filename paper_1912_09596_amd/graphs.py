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
