"""Brick-size autotuning: pick the brick edge B (8, 16 or 32 voxels) that
minimises the time of one TF change plus a number of frames for a volume,
measured on the device with the caller's own TF, camera and image size.

Only scheduling and timing live here; every measured step runs in libesk's
kernels.  A candidate that the library rejects for the volume's shape (more
than 1024 bricks per axis) is skipped.
"""
from __future__ import annotations

import statistics

from . import Context, EskError, Kd


def tune_brick(vol, tf, cam, size, accel="lbvh", frames_per_tf=1, candidates=(8, 16, 32), kd=None, reps=3,
               value_range=(0.0, 1.0), device=0):
    """Returns (best_brick, {brick: {"rebuild_ms", "render_ms", "cost_ms"}}).

    cost = rebuild + frames_per_tf * render, each the median of `reps`
    measurements (rebuild: host clock around the rebuild and a
    synchronisation, which includes a k-d build on its own stream; render:
    device events)."""
    import torch
    W, H = size
    build = ("kd",) if accel in ("kd", "hybrid") else (accel,) if accel != "none" else ("grid",)
    kd = kd or Kd()
    out = torch.empty((H, W, 4), dtype=torch.float32, device=vol.device)
    stream = torch.cuda.current_stream(vol.device)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    results = {}
    for B in candidates:
        ctx = Context(device)
        try:
            ctx.set_volume(vol, B, value_range, max_tf=max(256, tf.shape[0]))
        except EskError:
            ctx.close()
            continue
        import time
        rebuild, render = [], []
        for _ in range(reps):
            torch.cuda.synchronize()
            t = time.perf_counter()
            ctx.set_tf(tf, build=build, kd=kd)
            ctx.sync()
            rebuild.append((time.perf_counter() - t) * 1e3)
            e0.record(stream)
            ctx.render(cam, W, H, accel=accel, out=out)
            e1.record(stream)
            torch.cuda.synchronize()
            render.append(e0.elapsed_time(e1))
        rb, rd = statistics.median(rebuild), statistics.median(render)
        results[B] = {"rebuild_ms": rb, "render_ms": rd, "cost_ms": rb + frames_per_tf * rd}
        ctx.close()
    if not results:
        raise EskError(-3, "no candidate brick size fits the volume")
    best = min(results, key=lambda b: results[b]["cost_ms"])
    return best, results
