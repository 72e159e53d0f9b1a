"""Benchmark: per-TF rebuild + 1080p render on the 512^3 float32 noise volume.

Workload (one step): bind the volume (brick min/max), set the next TF of a
100-TF sequence and rebuild the macrocell grid, the LBVH and the binned k-d
tree, then render 1920x1080 with each of the three (one esk_render_multi
call: the three frames run concurrently).  The camera orbits 3.6 degrees
per TF.  Inputs are synthetic (seeded fractal value noise, ~5 %
non-empty voxels, 16^3 bricks) and resident in HBM before timing starts.

Prints one JSON line.  ``value`` = rays rendered per second over the whole
step (Mrays/s, all three renders, rebuilds and the min/max pass included).
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

W, H = 1920, 1080
DIMS = (512, 512, 512)
BRICK = 16
KD = dict(halting=1, max_leaf=32, bins=4)
ACCELS = ("grid", "lbvh", "kd")
# algorithmic FP32 operations per composited sample (counted from the
# formulas: lattice t 3, point 6, trilinear 30, normalise 5, TF lerp 13,
# opacity correction 5, compositing 9)
FLOP_PER_SAMPLE = 71
# FP32 vector peak without packed math (the build turns packed FP32 off):
# 256 CUs x 2.4 GHz x one wave64 VALU instruction per cycle per CU x 64
# lanes x 2 FLOP per fused multiply-add
PEAK_FP32_TFLOPS = 78.6
# VALU issue peak: one wave64 instruction per cycle per CU
PEAK_VALU_WAVE_INSTR_PER_S = 256 * 2.4e9
ISSUE_FILE = os.path.join(ROOT, "profiles", "render_issue_noise512_1080p.md")
ACCEL_CODE = {"grid": 1, "lbvh": 2, "kd": 4}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_noise512_1080p.md")
RENDER_SRC = os.path.join(ROOT, "paper_1912_09596_amd", "csrc", "render.hip")


def measured_traffic(accel):
    """HBM bytes per launch of k_render<accel> (f32 volume) from the committed
    FETCH_SIZE / WRITE_SIZE summary, or None when there is none or when the
    render source has changed since the counters were taken."""
    import hashlib
    try:
        text = open(TRAFFIC_FILE).read()
        src = hashlib.sha256(open(RENDER_SRC, "rb").read()).hexdigest()
    except OSError:
        return None
    if f"render.hip sha256: {src}" not in text:
        return None
    key = f"`k_render<{ACCEL_CODE[accel]}, float, unsigned int, true>`"
    for line in text.splitlines():
        cells = [c.strip() for c in line.strip().strip("|").split("|")]
        if cells and cells[0] == key:
            return int(float(cells[-1]))
    return None


def measured_issue(accel):
    """Per-launch counters of k_render<accel> (f32 volume) from the committed
    SQ/TCC summary: VALU instructions, lane instructions per composited
    sample, VALU issue and L2 figures; None when there is none or when the
    render source has changed since the counters were taken."""
    import hashlib
    try:
        text = open(ISSUE_FILE).read()
        src = hashlib.sha256(open(RENDER_SRC, "rb").read()).hexdigest()
    except OSError:
        return None
    if f"render.hip sha256: {src}" not in text:
        return None
    key = f"`k_render<{ACCEL_CODE[accel]}, float, unsigned int, true>`"
    header = None
    for line in text.splitlines():
        cells = [c.strip() for c in line.strip().strip("|").split("|")]
        if cells and cells[0] == "kernel":
            header = cells
        elif header and cells and cells[0] == key:
            return {h: float(v) for h, v in zip(header[1:], cells[1:])}
    return None


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    i = min(len(xs) - 1, max(0, int(round(q / 100.0 * (len(xs) - 1)))))
    return xs[i]


def host_cpu():
    """What the oracle runs on: logical CPUs, model, threads per core."""
    info = {"nproc": os.cpu_count(), "model": None, "threads_per_core": None}
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                info["model"] = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        siblings = open("/sys/devices/system/cpu/cpu0/topology/thread_siblings_list").read().strip()
        n = 0
        for part in siblings.split(","):
            a, _, b = part.partition("-")
            n += int(b) - int(a) + 1 if b else 1
        info["threads_per_core"] = n
    except (OSError, ValueError):
        pass
    return info


def cpu_baseline(vol, tfs, steps=3, stride=1, single_stride=64):
    """The CPU oracle on this host: `steps` steps of the same workload (min/max,
    classification, LBVH, k-d, and the three renders as full-march FP64
    images of every `stride`-th pixel of the 1080p frame) on all OpenMP
    threads; then one full-march render of every `single_stride`-th pixel
    on one thread and on all."""
    import numpy as np

    import oracle
    import synth

    L = oracle.lib()
    threads = L.orc_threads()
    nb = oracle.brick_grid(DIMS, BRICK)

    def run(nsteps, pstride):
        idx = np.arange(0, W * H, pstride)
        pix = np.stack([idx % W, idx // W], 1).astype(np.int32)
        rays = 0
        t0 = time.perf_counter()
        for j in range(nsteps):
            tf, cam = tfs[j], synth.c2_camera(j)
            mn, mx = oracle.brick_minmax(vol, BRICK)
            flags = oracle.classify(mn, mx, vol.dtype, tf)
            ids = oracle.compact(flags)
            k, i = oracle.sort_pairs(oracle.morton_keys(ids, nb[0], nb[1]), ids)
            oracle.lbvh(k, i, BRICK, DIMS)
            oracle.kd(flags, BRICK, DIMS, KD["halting"], KD["max_leaf"], KD["bins"])
            for _ in ACCELS:
                oracle.render(vol, tf, cam, W, H, 0.5, 1.0, pixels=pix)
                rays += pix.shape[0]
        return rays, time.perf_counter() - t0, pix.shape[0]

    rays, dt, npix = run(steps, stride)
    # the full-march render alone on one thread and on all, over the same
    # pixel subset (the per-step min/max and hierarchy builds left out)
    idx = np.arange(0, W * H, single_stride)
    pix1 = np.stack([idx % W, idx // W], 1).astype(np.int32)
    tf0, cam0 = tfs[0], synth.c2_camera(0)

    def render_rate():
        t = time.perf_counter()
        oracle.render(vol, tf0, cam0, W, H, 0.5, 1.0, pixels=pix1)
        return pix1.shape[0] / (time.perf_counter() - t) / 1e6

    r_all = render_rate()
    L.orc_set_threads(1)
    try:
        r_one = render_rate()
    finally:
        L.orc_set_threads(threads)
    host = host_cpu()
    return {"value": rays / dt / 1e6, "unit": "Mrays/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{steps} steps of the same workload (min/max, classify, LBVH, k-d, three "
                      f"full-march FP64 renders of {npix} of the 1920x1080 pixels each; "
                      f"{rays} rays) in {dt:.1f} s on {threads} OpenMP threads",
            "host": host,
            "render_only": {"unit": "Mrays/s", "one_thread": round(r_one, 4), "all_threads": round(r_all, 4),
                            "sample": f"one full-march FP64 render of every {single_stride}th pixel "
                                      f"({pix1.shape[0]} rays), TF 0, camera 0"}}


def batched_vs_plain(esk, torch, count=64, reps=5):
    """Many uneven volumes, each with its own TF and camera, 512x512 each:
    the plain path (one request at a time: rebuild, render, wait) against the
    batched path (one batched rebuild launch chain, one batched render
    launch, one wait), eager and captured in a graph.  All produce
    bit-identical images (checked)."""
    import numpy as np

    import synth

    reqs = synth.batch_workload(count)
    ctxs, tfs = [], []
    for r in reqs:
        c = esk.Context(0)
        brick = 8 if max(r["dims"]) <= 128 else 16
        c.set_volume(r["vol"], brick, (0.0, 1.0), max_tf=256)
        ctxs.append(c)
        tfs.append(torch.from_numpy(r["tf"]).cuda())
    cams = [r["cam"] for r in reqs]
    sizes = [(r["W"], r["H"]) for r in reqs]
    outs_p = [torch.empty((h, w, 4), dtype=torch.float32, device="cuda") for (w, h) in sizes]
    outs_b = [torch.empty((h, w, 4), dtype=torch.float32, device="cuda") for (w, h) in sizes]
    args = None

    def plain():
        for c, tf, cam, (w, h), o in zip(ctxs, tfs, cams, sizes, outs_p):
            c.set_tf(tf, build=("lbvh",))
            c.render(cam, w, h, accel="lbvh", out=o)
            torch.cuda.synchronize()

    rargs = None

    def batched():
        nonlocal args, rargs
        rargs = esk.rebuild_batch(ctxs, tfs, build=("lbvh",), args_buffer=rargs)
        esk.render_batch(ctxs, cams, sizes, accel="lbvh", outs=outs_b, args_buffer=args)
        args = ctxs[0]._keep["batch_args"]
        torch.cuda.synchronize()

    def rebuild_plain():
        for c, tf in zip(ctxs, tfs):
            c.set_tf(tf, build=("lbvh",))
        torch.cuda.synchronize()

    def rebuild_batched():
        esk.rebuild_batch(ctxs, tfs, build=("lbvh",), args_buffer=rargs)
        torch.cuda.synchronize()

    def render_plain():
        for c, cam, (w, h), o in zip(ctxs, cams, sizes, outs_p):
            c.render(cam, w, h, accel="lbvh", out=o)
        torch.cuda.synchronize()

    def render_batched():
        esk.render_batch(ctxs, cams, sizes, accel="lbvh", outs=outs_b, args_buffer=args)
        torch.cuda.synchronize()

    def timed(fn):
        fn()
        ts = []
        for _ in range(reps):
            t = time.perf_counter()
            fn()
            ts.append(time.perf_counter() - t)
        return statistics.median(ts)

    rays = sum(w * h for (w, h) in sizes)
    tp, tb = timed(plain), timed(batched)
    rp, rb = timed(render_plain), timed(render_batched)
    kp, kb = timed(rebuild_plain), timed(rebuild_batched)
    same = all(np.array_equal(a.cpu().numpy(), b.cpu().numpy()) for a, b in zip(outs_p, outs_b))
    for c in ctxs:
        c.close()

    # the batched rebuild + render captured into one graph, replayed with the
    # TFs refilled (one copy, one graph launch per batch)
    from paper_1912_09596_amd.graphs import BatchRebuildRenderGraph
    bricks = [8 if max(r["dims"]) <= 128 else 16 for r in reqs]
    g = BatchRebuildRenderGraph([r["vol"] for r in reqs], bricks, 256, cams, sizes, accel="lbvh")
    tf_stack = torch.stack(tfs)

    def graph_batched():
        g.replay(tf_stack)
        torch.cuda.synchronize()

    tg = timed(graph_batched)
    same_graph = all(torch.equal(a, b) for a, b in zip(g.outs, outs_p))
    g.close()

    # the same batch with brick sizes chosen per volume by the autotuner
    # (rebuild + one frame, on each request's own TF and camera); images do
    # not depend on the brick size, so they must equal the plain ones
    from paper_1912_09596_amd.tune import tune_brick
    t_tune = time.perf_counter()
    chosen = [tune_brick(r["vol"], tf, r["cam"], (r["W"], r["H"]), accel="lbvh", reps=2)[0]
              for r, tf in zip(reqs, tfs)]
    tune_s = time.perf_counter() - t_tune
    ctxs = []
    for r, B in zip(reqs, chosen):
        c = esk.Context(0)
        c.set_volume(r["vol"], B, (0.0, 1.0), max_tf=256)
        ctxs.append(c)
    args = None
    tt = timed(batched)
    rt = timed(render_batched)
    same_tuned = all(np.array_equal(a.cpu().numpy(), b.cpu().numpy()) for a, b in zip(outs_p, outs_b))
    for c in ctxs:
        c.close()
    return {"requests": count, "image": list(sizes[0]), "accel": "lbvh",
            "volumes": "axis sizes from {32..512}, u8 blobs at 1-20% density, own TF and camera each",
            "plain_mrays_per_s": round(rays / tp / 1e6, 1), "batched_mrays_per_s": round(rays / tb / 1e6, 1),
            "speedup": round(tp / tb, 3),
            "render_only": {"plain_mrays_per_s": round(rays / rp / 1e6, 1),
                            "batched_mrays_per_s": round(rays / rb / 1e6, 1), "speedup": round(rp / rb, 3)},
            "rebuild_only": {"plain_ms": round(kp * 1e3, 3), "batched_ms": round(kb * 1e3, 3),
                             "speedup": round(kp / kb, 3)},
            "graph": {"batched_mrays_per_s": round(rays / tg / 1e6, 1), "speedup_vs_eager_batched": round(tb / tg, 3),
                      "images_identical": bool(same_graph)},
            "images_identical": bool(same),
            "tuned_bricks": {"rule": "8^3 up to 128 voxels per axis, else 16^3 (above); tuned: per volume, "
                                     "the brick of {8,16,32} minimising rebuild + one frame",
                             "chosen": {str(b): chosen.count(b) for b in sorted(set(chosen))},
                             "tuning_s": round(tune_s, 2),
                             "batched_mrays_per_s": round(rays / tt / 1e6, 1),
                             "render_only_batched_mrays_per_s": round(rays / rt / 1e6, 1),
                             "images_identical": bool(same_tuned)}}


def graph_replay(esk, torch, count=200):
    """Launch-bound requests: a 64^3 u8 volume rendered at 256x256 with the
    LBVH, rebuilt for a new TF before every frame; eager calls against one
    HIP graph holding the rebuild and the render (replayed with the TF
    buffer refilled); then sixteen such requests per launch: plain calls,
    the batched calls, and the batched calls in one graph.  Requests per
    second, issued back to back."""
    import synth
    from paper_1912_09596_amd.graphs import RebuildRenderGraph

    w = synth.c1_workload()
    vol = torch.from_numpy(w["vol"]).cuda()
    cam = synth.perspective((64, 64, 64), 256, 256, synth.view_direction(3))
    tfs = [torch.from_numpy(synth.tf_random(500 + i, 256)).cuda() for i in range(8)]
    ctx = esk.Context(0)
    ctx.set_volume(vol, 8, max_tf=256)
    out = torch.empty((256, 256, 4), dtype=torch.float32, device="cuda")

    def eager(n):
        for i in range(n):
            ctx.set_tf(tfs[i % 8], build=("lbvh",))
            ctx.render(cam, 256, 256, accel="lbvh", out=out)
        torch.cuda.synchronize()

    g = RebuildRenderGraph(vol, 8, 256, cam, (256, 256), accel="lbvh")

    def graph(n):
        for i in range(n):
            g.replay(tfs[i % 8])
        torch.cuda.synchronize()

    res = {}
    for name, fn in (("eager", eager), ("graph", graph)):
        fn(20)
        t = time.perf_counter()
        fn(count)
        res[name + "_requests_per_s"] = round(count / (time.perf_counter() - t), 1)
    res["speedup"] = round(res["graph_requests_per_s"] / res["eager_requests_per_s"], 3)
    res["workload"] = "64^3 u8 blobs, 8^3 bricks, LBVH rebuild + 256x256 render per request"
    g.close()
    ctx.close()

    # the same requests sixteen at a time: plain calls, the batched calls,
    # and the batched calls captured in one graph
    from paper_1912_09596_amd.graphs import BatchRebuildRenderGraph
    nb = 16
    ctxs = []
    for _ in range(nb):
        c = esk.Context(0)
        c.set_volume(vol, 8, max_tf=256)
        ctxs.append(c)
    outs = [torch.empty((256, 256, 4), dtype=torch.float32, device="cuda") for _ in range(nb)]
    stacks = [torch.stack([tfs[(k + i) % 8] for i in range(nb)]) for k in range(8)]
    gb = BatchRebuildRenderGraph([vol] * nb, [8] * nb, 256, [cam] * nb, [(256, 256)] * nb, accel="lbvh")
    bufs = {}

    def plain16(n):
        for k in range(n):
            for i, c in enumerate(ctxs):
                c.set_tf(tfs[(k + i) % 8], build=("lbvh",))
                c.render(cam, 256, 256, accel="lbvh", out=outs[i])
        torch.cuda.synchronize()

    def batched16(n):
        for k in range(n):
            bufs["r"] = esk.rebuild_batch(ctxs, list(stacks[k % 8].unbind(0)), build=("lbvh",),
                                          args_buffer=bufs.get("r"))
            esk.render_batch(ctxs, [cam] * nb, [(256, 256)] * nb, accel="lbvh", outs=outs,
                             args_buffer=bufs.get("b"))
            bufs["b"] = ctxs[0]._keep["batch_args"]
        torch.cuda.synchronize()

    def graph16(n):
        for k in range(n):
            gb.replay(stacks[k % 8])
        torch.cuda.synchronize()

    b16 = {}
    for name, fn in (("plain", plain16), ("batched", batched16), ("graph", graph16)):
        fn(3)
        t = time.perf_counter()
        fn(count // nb)
        b16[name + "_requests_per_s"] = round((count // nb) * nb / (time.perf_counter() - t), 1)
    b16["graph_vs_plain"] = round(b16["graph_requests_per_s"] / b16["plain_requests_per_s"], 3)
    b16["graph_vs_batched"] = round(b16["graph_requests_per_s"] / b16["batched_requests_per_s"], 3)
    res["sixteen_per_launch"] = b16
    gb.close()
    for c in ctxs:
        c.close()
    return res


def small_config(esk, torch, reps=20):
    """The small configuration (64^3 u8 blobs, 8^3 bricks, 128x128, step 0.5):
    set_volume, each rebuild from enqueue to completion (wall clock, with the
    synchronisation), each render (HIP events); next to the latency floor of
    one tiny kernel launch waited on the same way."""
    import synth
    w = synth.c1_workload()
    vol = torch.from_numpy(w["vol"]).cuda()
    tf = torch.from_numpy(w["tf"]).cuda()
    ctx = esk.Context(0)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def wall(fn):
        ts = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - t) * 1e3)
        return round(statistics.median(ts), 4)

    res = {"workload": "64^3 u8 blobs (~10% non-zero), 8^3 bricks, ramp TF, 128x128 perspective, step 0.5"}
    res["set_volume_ms"] = wall(lambda: ctx.set_volume(vol, w["brick"], max_tf=256))
    res["rebuild_ms"] = {a: wall(lambda a=a: ctx.set_tf(tf, build=(a,), kd=esk.Kd(1, 32, 4)) or ctx.sync())
                         for a in ACCELS}
    ctx.set_tf(tf, build=ACCELS, kd=esk.Kd(1, 32, 4))
    out = torch.empty((w["H"], w["W"], 4), dtype=torch.float32, device="cuda")
    render = {}
    for a in ACCELS + ("none",):
        ts = []
        for _ in range(reps):
            e0.record(stream)
            ctx.render(w["cam"], w["W"], w["H"], accel=a, step=w["dt"], out=out)
            e1.record(stream)
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        render[a] = round(statistics.median(ts), 4)
    res["render_ms"] = render
    res["render_mrays_per_s"] = {a: round(w["W"] * w["H"] / render[a] / 1e3, 1) for a in render}
    x = torch.zeros(1, device="cuda")
    res["launch_floor_ms"] = wall(lambda: x.add_(1.0))
    ctx.close()
    return res


def large_volumes(esk, torch, reps=3):
    """1024^3 tubes (~2 % of voxels) stored as f32 and f16, 2048^3 tubes stored
    as u16, 8^3 bricks: set_volume, rebuild per structure and 1080p render
    per structure (perspective).  Errors against the oracle are checked by
    the test suite on sampled pixels; here only times are taken."""
    import synth

    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    stream = torch.cuda.current_stream()

    def ev_ms(fn):
        times = []
        for _ in range(reps):
            e0.record(stream)
            fn()
            e1.record(stream)
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
        return round(statistics.median(times), 4)

    out = {}
    kd = esk.Kd(**KD)
    for w in synth.c3_workloads():
        dims = w["dims"]
        src = synth.tubes_torch(dims, w["fraction"], w["seed"])
        tf = torch.from_numpy(synth.tf_random(w["seed"], 256)).cuda()
        cam = synth.perspective(dims, W, H, synth.view_direction(w["seed"]))
        for storage in w["storage"]:
            if storage == "f32":
                dv = src
            elif storage == "f16":
                dv = src.to(torch.float16)
            else:
                q = torch.empty(src.shape, dtype=torch.int16, device=src.device)
                for z in range(0, src.shape[0], 128):
                    q[z:z + 128] = torch.floor(src[z:z + 128] * 65535.0 + 0.5).to(torch.int32).to(torch.int16)
                dv = q.view(torch.uint16)
            ctx = esk.Context(0)
            ctx.set_volume(dv, 8, (0.0, 1.0), max_tf=256)
            rec = {"dims": list(dims), "storage": storage, "brick": 8,
                   "set_volume_ms": ev_ms(lambda: ctx.set_volume(dv, 8, (0.0, 1.0), max_tf=256,
                                                                 workspace=ctx._keep["ws"]))}
            rebuild = {}
            for a in ACCELS:
                times = []
                for _ in range(reps):
                    torch.cuda.synchronize()
                    t = time.perf_counter()
                    ctx.set_tf(tf, build=(a,), kd=kd)
                    ctx.sync()   # every structure complete (see the phase breakdown)
                    torch.cuda.synchronize()
                    times.append((time.perf_counter() - t) * 1e3)
                rebuild[a] = round(statistics.median(times), 4)
            ctx.set_tf(tf, build=ACCELS, kd=kd)
            img = torch.empty((H, W, 4), dtype=torch.float32, device="cuda")
            render = {a: ev_ms(lambda a=a: ctx.render(cam, W, H, accel=a, out=img)) for a in ACCELS + ("none",)}
            st = ctx.stats()
            ctx.set_tf(tf, build=("kd",), kd=esk.Kd(0, 0, 4))
            for a in ("kd", "hybrid"):
                render[a + "_shallow"] = ev_ms(lambda a=a: ctx.render(cam, W, H, accel=a, out=img))
            rec.update({"rebuild_ms": rebuild, "render_ms": render,
                        "render_mrays_per_s": {a: round(W * H / v / 1e3, 1) for a, v in render.items()},
                        "bricks_nonempty": st["n_nonempty"], "bricks": st["n_bricks"],
                        "lbvh_nodes": st["lbvh_nodes"], "kd_nodes": st["kd_nodes"], "kd_height": st["kd_height"]})
            out[f"{w['name']}_{storage}"] = rec
            ctx.close()
            del dv, ctx
            torch.cuda.empty_cache()
        del src
        torch.cuda.empty_cache()
    return out


def statistics_table(esk, torch, noise_vol, reps=3):
    """Node counts, heights and rebuild times of the LBVH and of the k-d
    variants (shallow, deep, deep + MLS 32, deep + MLS 128; 4 bins), each
    with the brick-tight and the voxel-tight split cost, on the synthetic
    stand-ins, 8^3 bricks, one ramp TF (alpha > 0 above s = 0.02): the
    quantities of the paper's statistics table (Sec. 4.3)."""
    import numpy as np

    import synth

    rng = np.random.default_rng(7)
    tf = torch.from_numpy(synth.tf_ramp(256, start=0.02)).cuda()
    variants = {"shallow": esk.Kd(0, 0, 4), "deep": esk.Kd(1, 0, 4), "deep_mls32": esk.Kd(1, 32, 4),
                "deep_mls128": esk.Kd(1, 128, 4)}
    cases = [("blobs256_u8", lambda: synth._blob_volume_torch((256, 256, 256), 8, 0.1, rng, "cuda", "u8")),
             ("noise512_f32", lambda: noise_vol),
             ("tubes1024_f32", lambda: synth.tubes_torch((1024, 1024, 1024), 0.02, 31)),
             ("menger243_u8", lambda: torch.from_numpy(synth.menger_sponge(4, 3)).cuda())]

    def timed(ctx, build, kd=None, kd_cost="brick"):
        times = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t = time.perf_counter()
            ctx.set_tf(tf, build=build, kd=kd, kd_cost=kd_cost)
            ctx.sync()   # every structure complete (see the phase breakdown)
            torch.cuda.synchronize()
            times.append((time.perf_counter() - t) * 1e3)
        return round(statistics.median(times), 4)

    out = {}
    for name, make in cases:
        vol = make()
        ctx = esk.Context(0)
        ctx.set_volume(vol, 8, (0.0, 1.0), max_tf=256)
        rec = {"dims": list(vol.shape[::-1]), "grid_ms": timed(ctx, ("grid",))}
        ms = timed(ctx, ("lbvh",))
        st = ctx.stats()
        rec.update({"bricks": st["n_bricks"], "bricks_nonempty": st["n_nonempty"],
                    "lbvh": {"nodes": st["lbvh_nodes"], "height": st["lbvh_height"], "rebuild_ms": ms}})
        for vname, kd in variants.items():
            ms = timed(ctx, ("kd",), kd)
            st = ctx.stats()
            rec[f"kd_{vname}"] = {"nodes": st["kd_nodes"], "height": st["kd_height"], "rebuild_ms": ms}
            # the voxel-tight split cost (Sec. 3.2.2): same rules, union volumes
            # of the bricks' voxel-tight boxes (the rebuild includes those boxes)
            ms = timed(ctx, ("kd",), kd, kd_cost="tight")
            st = ctx.stats()
            rec[f"kd_{vname}_tight_cost"] = {"nodes": st["kd_nodes"], "height": st["kd_height"], "rebuild_ms": ms}
        out[name] = rec
        ctx.close()
        del vol, ctx
        torch.cuda.empty_cache()
    return out


def sort_paths(esk, torch, reps=5):
    """The sorted Morton keys of the LBVH rebuild (Sec. 3.1) by LSD radix sort
    on a lopsided brick grid (4096x256x128 u8, 8^3 bricks: 512x32x16 bricks,
    code domain 2^27 >> 4x the brick count) next to the Morton enumeration on
    a cube with the same brick count (512^3 u8, 64^3 bricks), both ~10 %
    blob voxels.  Per case: grid rebuild (classification only) and LBVH
    rebuild from enqueue to completion; their difference is the sorted keys,
    the Karras nodes and the boxes."""
    import numpy as np

    import synth

    tf = torch.from_numpy(synth.tf_ramp(256, start=0.02)).cuda()
    cases = [("lopsided_4096x256x128_u8", (4096, 256, 128), 64, "radix sort"),
             ("cube_512_u8", (512, 512, 512), 8, "Morton enumeration")]

    def timed(ctx, build):
        times = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t = time.perf_counter()
            ctx.set_tf(tf, build=build)
            torch.cuda.synchronize()
            times.append((time.perf_counter() - t) * 1e3)
        return round(statistics.median(times), 4)

    out = {}
    for name, dims, blobs, path in cases:
        rng = np.random.default_rng(11)
        vol = synth._blob_volume_torch(dims, blobs, 0.1, rng, "cuda", "u8")
        ctx = esk.Context(0)
        ctx.set_volume(vol, 8, (0.0, 1.0), max_tf=256)
        g = timed(ctx, ("grid",))
        lb = timed(ctx, ("lbvh",))
        st = ctx.stats()
        out[name] = {"dims": list(dims), "bricks": st["n_bricks"], "bricks_nonempty": st["n_nonempty"],
                     "sorted_keys_by": path, "grid_rebuild_ms": g, "lbvh_rebuild_ms": lb,
                     "keys_nodes_boxes_ms": round(lb - g, 4)}
        ctx.close()
        del vol, ctx
        torch.cuda.empty_cache()
    return out


def serving(esk, torch, n_req=400, rate=200.0, seed=6):
    """A Poisson stream of TF edits and renders over 16 resident volumes
    (128^3..1024^3, u8 and f16), images 256^2..1920x1080: continuous
    batching (paper_1912_09596_amd.serve) against serving one request at a
    time on arrival, at the stream's rate and with every request queued at
    t = 0 (saturation)."""
    import numpy as np

    import synth
    from paper_1912_09596_amd.serve import Request, Server

    vols = synth.serving_volumes(16)
    tfs = [torch.from_numpy(synth.tf_random(seed * 100 + i, 256)).cuda() for i in range(32)]
    srv = Server(hbm_budget_bytes=64 << 30, max_batch=32)
    for v in vols:
        srv.add_volume(v["name"], v["vol"], 16 if v["dims"][0] >= 512 else 8, tf=torch.from_numpy(v["tf"]).cuda())
    sizes = [(256, 256), (512, 512), (1280, 720), (1920, 1080)]

    def make(r, zero=False):
        rng = np.random.default_rng(seed)
        reqs, t = [], 0.0
        for rid in range(n_req):
            t += rng.exponential(1.0 / r)
            v = vols[int(rng.integers(0, len(vols)))]
            at = 0.0 if zero else t
            if rng.random() < 0.3:
                reqs.append(Request(rid, v["name"], "rebuild", at, tf=tfs[int(rng.integers(0, len(tfs)))]))
            else:
                W, H = sizes[int(rng.integers(0, len(sizes)))]
                cam = synth.perspective(v["dims"], W, H, synth.view_direction(seed * 1000 + rid))
                reqs.append(Request(rid, v["name"], "render", at, cam=cam, size=(W, H)))
        return reqs

    def plain(reqs):
        outs = {}
        t0 = time.perf_counter()
        for r in sorted(reqs, key=lambda q: (q.arrival, q.rid)):
            while time.perf_counter() - t0 < r.arrival:
                pass
            c = srv.contexts[r.volume]
            if r.kind == "rebuild":
                c.set_tf(r.tf, build=("lbvh",))
            else:
                outs[r.rid] = c.render(r.cam, r.size[0], r.size[1], accel="lbvh")
            torch.cuda.synchronize()
            r.done = time.perf_counter() - t0
        return Server._summary(reqs, time.perf_counter() - t0), outs

    init_tfs = {v["name"]: torch.from_numpy(v["tf"]).cuda() for v in vols}

    def reset():
        for name, tf in init_tfs.items():
            srv.contexts[name].set_tf(tf, build=("lbvh",))
        torch.cuda.synchronize()

    def fmt(st):
        return {k: (round(v, 3) if isinstance(v, float) else v) for k, v in st.items()}

    out = {"volumes": "16 resident cubes 128^3..1024^3, u8 and f16 alternating, blob sums at 1-20% density",
           "requests": n_req, "mix": "30% TF edits (LBVH rebuild), 70% renders 256^2..1920x1080", "accel": "lbvh"}
    # warm up both paths once
    srv.run(make(rate * 10, zero=True)[:32])
    plain(make(rate * 10, zero=True)[:32])
    for label, zero in (("poisson_200_per_s", False), ("saturated", True)):
        reset()
        reqs = make(rate, zero)
        st_s = srv.run(reqs)
        served_out = {r.rid: r.out for r in reqs if r.kind == "render"}
        reset()
        reqs_p = make(rate, zero)
        st_p, plain_out = plain(reqs_p)
        same = all(torch.equal(served_out[k], plain_out[k]) for k in plain_out)
        out[label] = {"served": fmt(st_s), "one_at_a_time": fmt(st_p), "results_identical": bool(same)}
    return out


# --------------------------------------------------------------------------
# profile summaries (no GPU): markdown tables from rocprofv3 result databases
# --------------------------------------------------------------------------

def _short_kernel(name):
    short = name.replace("esk::(anonymous namespace)::", "").replace("void ", "")
    short = short.split("(esk::")[0].split("(float const*")[0].split("(unsigned int*")[0]
    if "at::native" in short:
        short = short.split("<")[0] + " (torch)"
    return short


def trace_markdown(db, command):
    """Kernel-trace table (calls, total and average duration, resources)."""
    import sqlite3
    c = sqlite3.connect(db)
    rows = list(c.execute("select name, total_calls, total_duration, average, percentage from top_kernels"))
    regs = {r[0]: r[1:] for r in c.execute("select name, vgpr_count, sgpr_count, lds_size, scratch_size from kernels")}
    out = ["# Kernel trace: 512^3 f32 noise volume, 1920x1080, grid + LBVH + k-d per TF", "",
           "Command (from the repository root on the MI355X box):", "", "```", command, "```", "",
           "| kernel | calls | total ms | avg us | % | VGPR | SGPR | LDS B | scratch B |",
           "|---|---:|---:|---:|---:|---:|---:|---:|---:|"]
    for name, n, tot, avg, pct in rows:
        if pct < 0.05:
            continue
        r = regs.get(name, ("", "", "", ""))
        # the view reports durations in microseconds
        out.append(f"| `{_short_kernel(name)[:70]}` | {n} | {tot / 1e3:.2f} | {avg:.1f} | {pct:.1f} | "
                   f"{r[0]} | {r[1]} | {r[2]} | {r[3]} |")
    return "\n".join(out)


def ranges_markdown(db, command):
    """Host time of the library's entry points from a rocprofv3 --marker-trace
    database (the named ranges each entry point opens): calls, median, 90th
    percentile and maximum in microseconds."""
    import collections
    import json as _json
    import sqlite3
    c = sqlite3.connect(db)
    per = collections.defaultdict(list)
    for ext, dur in c.execute("select extdata, duration from regions where category like 'MARKER%'"):
        try:
            name = _json.loads(ext or "{}").get("message", "")
        except ValueError:
            name = ""
        if name.startswith("esk_"):
            per[name].append(dur / 1e3)
    out = ["# Host time per entry point: 512^3 f32 noise volume, 1920x1080, grid + LBVH + k-d per TF", "",
           "Command (from the repository root on the MI355X box):", "", "```", command, "```", "",
           "Each entry point opens a named host range (roctx) for its duration: argument checks, "
           "enqueueing its kernels and copies, and any wait it makes (esk_sync waits for the device).  "
           "The first calls include allocations and module loading.", "",
           "| entry point | calls | median us | p90 us | max us |", "|---|---:|---:|---:|---:|"]
    for name in sorted(per, key=lambda n: -sum(per[n])):
        v = sorted(per[name])
        p90 = v[min(len(v) - 1, int(0.9 * len(v)))]
        out.append(f"| `{name}` | {len(v)} | {statistics.median(v):.1f} | {p90:.1f} | {v[-1]:.1f} |")
    return "\n".join(out)


def counters_markdown(fetch_db, write_db, command):
    """HBM traffic per launch from FETCH_SIZE and WRITE_SIZE runs (KiB per
    dispatch), each scaled by what the counter reads for the 512 MiB device
    copy the runs start with (--copy-probe)."""
    import collections
    import hashlib
    import sqlite3

    def load(db, counter):
        c = sqlite3.connect(db)
        per = collections.defaultdict(list)
        for k, v in c.execute("select kernel_name, value from counters_collection where counter_name = ?",
                              (counter,)):
            per[k].append(v)
        return per

    fetch, write = load(fetch_db, "FETCH_SIZE"), load(write_db, "WRITE_SIZE")
    probe_kib = float(512 * 1024)
    copy_f = max(v for k, vs in fetch.items() if "copyBuffer" in k for v in vs)
    copy_w = max(v for k, vs in write.items() if "copyBuffer" in k for v in vs)
    sf, sw = probe_kib / copy_f, probe_kib / copy_w
    src = hashlib.sha256(open(RENDER_SRC, "rb").read()).hexdigest()
    out = ["# HBM traffic per launch: 512^3 f32 noise volume, 1920x1080, grid + LBVH + k-d per TF", "",
           "Commands (from the repository root on the MI355X box; one counter per run):", "", "```", command, "```",
           "", f"render.hip sha256: {src}", "",
           f"Copy probe (one plain 512 MiB device copy): FETCH_SIZE reads {copy_f:.0f} KiB, WRITE_SIZE "
           f"{copy_w:.0f} KiB of 524288 KiB moved, so FETCH_SIZE is scaled by {sf:.3f} and WRITE_SIZE by "
           f"{sw:.3f}.  Each row averages every dispatch of the kernel in the run: the timed steps, the "
           f"warm-up and the phase-breakdown renders (for the k-d and LBVH renders these include the shallow "
           f"tree and the voxel-tight variants).", "",
           "| kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | HBM bytes per launch |",
           "|---|---:|---:|---:|---:|"]
    for k in fetch:
        if k not in write or "copyBuffer" in k or "fillBuffer" in k:
            continue
        f = statistics.mean(fetch[k])
        w = statistics.mean(write[k])
        out.append(f"| `{_short_kernel(k)[:70]}` | {len(fetch[k])} | {f:.0f} | {w:.0f} | "
                   f"{int(round((f * sf + w * sw) * 1024))} |")
    return "\n".join(out)


ISSUE_COUNTERS_A = ["SQ_WAVES", "SQ_INSTS_VALU", "SQ_ACTIVE_INST_VALU", "SQ_INSTS_VMEM_RD", "SQ_INSTS_LDS",
                    "SQ_BUSY_CU_CYCLES", "SQ_WAVE_CYCLES", "SQ_WAIT_INST_ANY"]
ISSUE_COUNTERS_B = ["TCC_REQ_sum", "TCC_HIT_sum", "TCC_MISS_sum", "TCP_TCC_READ_REQ_sum", "TA_BUSY_avr",
                    "GRBM_GUI_ACTIVE"]


def profile_frames(reps=3):
    """The frame the render counters are taken on: the 512^3 noise volume
    with TF 0 and camera 0, each structure rebuilt once and rendered `reps`
    times at 1920x1080; prints the composited samples per structure."""
    import torch

    import paper_1912_09596_amd as esk
    import synth

    vol = synth.fractal_noise(DIMS, seed=2)
    tf = torch.from_numpy(synth.c2_tfs(1)[0]).cuda()
    cam = synth.c2_camera(0)
    ctx = esk.Context(0)
    ctx.set_volume(torch.from_numpy(vol).cuda(), BRICK, (0.0, 1.0), max_tf=256)
    ctx.set_tf(tf, build=ACCELS, kd=esk.Kd(**KD))
    out = torch.empty((H, W, 4), dtype=torch.float32, device="cuda")
    cnt = torch.empty((H, W), dtype=torch.int32, device="cuda")
    samples = {}
    for a in ACCELS + ("none",):
        for _ in range(reps):
            ctx.render(cam, W, H, accel=a, out=out)
        ctx.render(cam, W, H, accel=a, out=out, counts=cnt)
        samples[a] = int(cnt.sum().item())
    torch.cuda.synchronize()
    print(json.dumps({"frame": "512^3 noise, TF 0, camera 0, 1920x1080", "reps": reps, "samples": samples}))


def issue_markdown(db_a, db_b, frames_json, command):
    """Per-launch SQ / TCC / TA counters of the render kernels on the profiled
    frame (two rocprofv3 --pmc runs of the same command), with the VALU
    instructions per composited sample and the VALU issue rate."""
    import collections
    import hashlib
    import sqlite3

    def load(db):
        c = sqlite3.connect(db)
        per = collections.defaultdict(lambda: collections.defaultdict(list))
        for k, n, v in c.execute("select kernel_name, counter_name, value from counters_collection"):
            per[k][n].append(v)
        return per

    a, b = load(db_a), load(db_b)
    frames = json.load(open(frames_json))
    samples = frames["samples"]
    code = {v: k for k, v in ACCEL_CODE.items()}
    code[0] = "none"
    src = hashlib.sha256(open(RENDER_SRC, "rb").read()).hexdigest()
    out = ["# Render counters: 512^3 f32 noise volume, 1920x1080, TF 0 / camera 0", "",
           "Commands (from the repository root on the MI355X box; one counter set per run):", "", "```",
           command, "```", "", f"render.hip sha256: {src}", "",
           f"Frame: {frames['frame']}; every kernel rendered it {frames['reps'] + 1} times per run and each "
           "row averages those dispatches.  Composited samples per frame: " +
           ", ".join(f"{k} {v}" for k, v in samples.items()) + ".  "
           "`lane instr / sample` = SQ_INSTS_VALU x 64 / composited samples (for the skipping modes the "
           "samples of non-empty bricks, the grid's count).  `kernel cycles` = GRBM_GUI_ACTIVE / 8 (the "
           "counter adds up the 8 XCDs).  `VALU issue` = SQ_INSTS_VALU / (kernel cycles x 256 CUs): the "
           "fraction of the one-wave64-VALU-instruction-per-cycle-per-CU rate the kernel reached.  "
           "`L2 hit` = TCC_HIT / TCC_REQ.", "",
           "| kernel | dispatches | waves | VALU instr | lane instr / sample | VALU issue | VMEM rd instr | "
           "LDS instr | wait cycles | wave cycles | kernel cycles | L2 requests | L2 hit | TCP->L2 reads | "
           "TA busy |",
           "|---|" + "---:|" * 14]
    for k in sorted(a):
        if "k_render<" not in k or "float, unsigned int, true" not in k or k not in b:
            continue
        acc = int(_short_kernel(k).split("<")[1].split(",")[0])
        m = {n: statistics.mean(v) for n, v in a[k].items()}
        m.update({n: statistics.mean(v) for n, v in b[k].items()})
        ns = samples["grid"] if acc != 0 else samples["none"]
        lane = m["SQ_INSTS_VALU"] * 64 / ns
        cycles = m["GRBM_GUI_ACTIVE"] / 8
        issue = m["SQ_INSTS_VALU"] / (cycles * 256)
        hit = m["TCC_HIT_sum"] / max(1.0, m["TCC_REQ_sum"])
        out.append(f"| `{_short_kernel(k)[:70]}` | {len(a[k]['SQ_INSTS_VALU'])} | {m['SQ_WAVES']:.0f} | "
                   f"{m['SQ_INSTS_VALU']:.0f} | {lane:.1f} | {issue:.3f} | {m['SQ_INSTS_VMEM_RD']:.0f} | "
                   f"{m['SQ_INSTS_LDS']:.0f} | {m['SQ_WAIT_INST_ANY']:.0f} | {m['SQ_WAVE_CYCLES']:.0f} | "
                   f"{cycles:.0f} | {m['TCC_REQ_sum']:.0f} | {hit:.3f} | "
                   f"{m['TCP_TCC_READ_REQ_sum']:.0f} | {m['TA_BUSY_avr']:.0f} |")
    return "\n".join(out)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-large", action="store_true", help="skip the 1024^3 / 2048^3 storage-precision section")
    ap.add_argument("--no-stats", action="store_true", help="skip the node/height statistics table")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run one plain 512 MiB device copy first (reference for HBM counters)")
    ap.add_argument("--trace-md", nargs=2, metavar=("DB", "COMMAND"),
                    help="print the kernel-trace summary of a rocprofv3 database and exit")
    ap.add_argument("--counters-md", nargs=3, metavar=("FETCH_DB", "WRITE_DB", "COMMAND"),
                    help="print the HBM traffic summary of two rocprofv3 --pmc databases and exit")
    ap.add_argument("--ranges-md", nargs=2, metavar=("DB", "COMMAND"),
                    help="print the host time per entry point from a rocprofv3 --marker-trace database and exit")
    ap.add_argument("--profile-frames", action="store_true",
                    help="render the profiled frame with every structure (for rocprofv3 --pmc runs) and exit")
    ap.add_argument("--issue-md", nargs=4, metavar=("DB_A", "DB_B", "FRAMES_JSON", "COMMAND"),
                    help="print the render counter summary of two rocprofv3 --pmc databases and exit")
    ap.add_argument("--cpu-steps", type=int, default=3)
    ap.add_argument("--cpu-stride", type=int, default=1)
    args = ap.parse_args()
    if args.trace_md:
        print(trace_markdown(*args.trace_md))
        return
    if args.ranges_md:
        print(ranges_markdown(*args.ranges_md))
        return
    if args.counters_md:
        print(counters_markdown(*args.counters_md))
        return
    if args.issue_md:
        print(issue_markdown(*args.issue_md))
        return
    if args.profile_frames:
        profile_frames()
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1912_09596_amd as esk
    import synth

    log("generating 512^3 noise volume and 100 TFs")
    vol = synth.fractal_noise(DIMS, seed=2)
    tfs = synth.c2_tfs(100)
    dev = torch.device("cuda", 0)
    dvol = torch.from_numpy(vol).to(dev)
    dtfs = [torch.from_numpy(t).to(dev) for t in tfs]
    cams = [synth.c2_camera(i) for i in range(100)]
    ctx = esk.Context(0)
    ws = torch.empty(esk.workspace_bytes(DIMS, esk.F32, BRICK, 256), dtype=torch.uint8, device=dev)
    outs = {a: torch.empty((H, W, 4), dtype=torch.float32, device=dev) for a in ACCELS}
    kd = esk.Kd(**KD)
    stream = torch.cuda.current_stream()

    # esk_render_multi runs the frames of the trees on the context's build
    # streams and the grid's on its own: events on a tree's stream around the
    # call bracket that tree's frame (esk_render_stream)
    tree_streams = {a: torch.cuda.ExternalStream(ctx.render_stream(a), device=dev) for a in ("lbvh", "kd")}

    def step(i, ev=None):
        j = i % 100
        ctx.set_volume(dvol, BRICK, (0.0, 1.0), max_tf=256, workspace=ws)
        ctx.set_tf(dtfs[j], build=ACCELS, kd=kd)
        if ev is not None:
            for a, s_ in tree_streams.items():
                ev[a][0].record(s_)
        ctx.render_multi([dict(cam=cams[j], W=W, H=H, accel=a, out=outs[a]) for a in ACCELS], step=0.5, ref=1.0)
        if ev is not None:
            for a, s_ in tree_streams.items():
                ev[a][1].record(s_)

    if args.copy_probe:
        src = torch.empty(128 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    log(f"warmup {args.warmup}")
    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()

    events = [{a: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for a in tree_streams} for _ in range(args.steps)]
    log(f"timing {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(args.warmup + i, events[i])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    # the trees' frames inside the timed steps, beside the other frames
    render_ms_step = {a: [events[i][a][0].elapsed_time(events[i][a][1]) for i in range(args.steps)]
                      for a in tree_streams}
    rays = len(ACCELS) * W * H * args.steps
    value = rays / elapsed / 1e6

    # each structure's frame alone (one esk_render on the context's stream),
    # over the TFs and cameras of the timed steps
    log("renders alone")
    render_ms = {a: [] for a in ACCELS}
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for i in range(args.steps):
        j = (args.warmup + i) % 100
        ctx.set_tf(dtfs[j], build=ACCELS, kd=kd)
        for a in ACCELS:
            e0.record(stream)
            ctx.render(cams[j], W, H, accel=a, step=0.5, ref=1.0, out=outs[a])
            e1.record(stream)
            torch.cuda.synchronize()
            render_ms[a].append(e0.elapsed_time(e1))

    # per-phase breakdown (outside the timed region)
    log("phase breakdown")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    sv = []
    for _ in range(5):
        e0.record(stream)
        ctx.set_volume(dvol, BRICK, (0.0, 1.0), max_tf=256, workspace=ws)
        e1.record(stream)
        torch.cuda.synchronize()
        sv.append(e0.elapsed_time(e1))
    rebuild = {}
    for a in ACCELS:
        times = []
        for i in range(min(args.steps, 100)):
            torch.cuda.synchronize()
            t = time.perf_counter()
            ctx.set_tf(dtfs[i % 100], build=(a,), kd=kd)
            # esk_sync: every structure complete (a k-d batch of level launches that fell short is finished)
            ctx.sync()
            torch.cuda.synchronize()
            times.append((time.perf_counter() - t) * 1e3)
        rebuild[a] = {"median_ms": statistics.median(times), "p99_ms": percentile(times, 99)}
    # samples per frame (composited) for the dominant-kernel roofline
    j = (args.warmup + args.steps - 1) % 100
    ctx.set_tf(dtfs[j], build=ACCELS, kd=kd)
    samples = {}
    cnt = torch.empty((H, W), dtype=torch.int32, device=dev)
    for a in ACCELS + ("none",):
        ctx.render(cams[j], W, H, accel=a, out=outs.get(a, outs["lbvh"]), counts=cnt)
        samples[a] = int(cnt.sum().item())
    naive = []
    for _ in range(3):
        e0.record(stream)
        ctx.render(cams[j], W, H, accel="none", out=outs["lbvh"])
        e1.record(stream)
        torch.cuda.synchronize()
        naive.append(e0.elapsed_time(e1))
    st = ctx.stats()
    # the hybrid grid (Sec. 3.3): a shallow k-d tree, the macrocell grid inside its leaves
    shallow = {}
    ctx.set_tf(dtfs[j], build=("kd",), kd=esk.Kd(0, 0, 4))
    for a in ("kd", "hybrid"):
        times = []
        for _ in range(3):
            e0.record(stream)
            ctx.render(cams[j], W, H, accel=a, out=outs["lbvh"])
            e1.record(stream)
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
        shallow[a + "_render_ms"] = round(statistics.median(times), 4)
    shallow["kd_nodes"] = ctx.stats()["kd_nodes"]
    # voxel-tight boxes (ESK_TIGHT_BOXES): rebuild of all three structures and
    # the tree renders with leaves marched inside the bricks' tight boxes
    tight = {}
    times = []
    for i in range(5):
        torch.cuda.synchronize()
        t = time.perf_counter()
        ctx.set_tf(dtfs[j], build=ACCELS, kd=kd, tight=True)
        ctx.sync()
        times.append((time.perf_counter() - t) * 1e3)
    tight["rebuild_all_ms"] = round(statistics.median(times), 4)
    times = []
    for i in range(5):
        torch.cuda.synchronize()
        t = time.perf_counter()
        ctx.set_tf(dtfs[j], build=("kd",), kd=kd, kd_cost="tight")
        ctx.sync()
        times.append((time.perf_counter() - t) * 1e3)
    tight["kd_tight_cost_rebuild_ms"] = round(statistics.median(times), 4)
    st_t = ctx.stats()
    tight["kd_tight_cost_nodes"], tight["kd_tight_cost_height"] = st_t["kd_nodes"], st_t["kd_height"]
    rt = []
    for _ in range(3):
        e0.record(stream)
        ctx.render(cams[j], W, H, accel="kd", out=outs["lbvh"])
        e1.record(stream)
        torch.cuda.synchronize()
        rt.append(e0.elapsed_time(e1))
    tight["kd_tight_cost_render_ms"] = round(statistics.median(rt), 4)
    ctx.set_tf(dtfs[j], build=ACCELS, kd=kd, tight=True)
    for a in ("lbvh", "kd"):
        rt = []
        for _ in range(3):
            e0.record(stream)
            ctx.render(cams[j], W, H, accel=a, out=outs["lbvh"])
            e1.record(stream)
            torch.cuda.synchronize()
            rt.append(e0.elapsed_time(e1))
        tight[a + "_render_ms"] = round(statistics.median(rt), 4)
        ctx.render(cams[j], W, H, accel=a, out=outs["lbvh"], counts=cnt)
        tight[a + "_samples"] = int(cnt.sum().item())

    # a plain device copy of the volume's size: the streaming rate this box
    # reaches, next to which set_volume's rate is read
    src = dvol.view(-1)
    dst = torch.empty_like(src)
    cp = []
    for _ in range(5):
        e0.record(stream)
        dst.copy_(src)
        e1.record(stream)
        torch.cuda.synchronize()
        cp.append(e0.elapsed_time(e1))
    del dst
    copy_gbs = 2 * src.numel() * 4 / (statistics.median(cp) * 1e-3) / 1e9
    # set_volume's algorithmic bytes (FP32, bricks of 16): the blocked copy
    # reads the volume once and writes the blocked layout (per 8^3 block its
    # 9^3 voxels, padded to 736 values) and 16 min/max summaries per block;
    # the bricks' min/max are combined from those and written
    nvox = DIMS[0] * DIMS[1] * DIMS[2]
    nblocks = ((DIMS[0] + 7) // 8) * ((DIMS[1] + 7) // 8) * ((DIMS[2] + 7) // 8)
    sv_bytes = nvox * 4 + nblocks * 736 * 4 + nblocks * 64 + 2 * st["n_bricks"] * 4
    sv_gbs = sv_bytes / (statistics.median(sv) * 1e-3) / 1e9

    mean_ms = {a: statistics.mean(render_ms[a]) for a in ACCELS}
    dominant = max(ACCELS, key=lambda a: mean_ms[a])
    # its launches inside the timed steps (on its own stream, beside the other frames)
    dom_ms = render_ms_step.get(dominant, render_ms[dominant])
    # algorithmic work of every timed step's frame: the samples of its
    # non-empty bricks (what the grid composites; trees may also march some
    # empty-brick samples, which do not count), counted after the timing
    step_samples = []
    for i in range(args.steps):
        j = (args.warmup + i) % 100
        ctx.set_tf(dtfs[j], build=("grid",))
        ctx.render(cams[j], W, H, accel="grid", out=outs["grid"], counts=cnt)
        step_samples.append(int(cnt.sum().item()))
    flops = sum(step_samples) * FLOP_PER_SAMPLE
    achieved = flops / (sum(dom_ms) * 1e-3) / 1e12
    issue = measured_issue(dominant)
    # a1's algorithmic bytes: the volume read once, the bricks' min/max written
    a1_bytes = nvox * 4 + 2 * st["n_bricks"] * 4
    result = {
        "metric": "Mrays/s at 1080p + rebuild ms per TF change; batched vs plain, RGBA err≤1e-3",
        "value": round(value, 2),
        "unit": "Mrays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "512^3 float32 fractal-noise volume (~5% non-empty), 16^3 bricks, "
                               "100-TF sequence, 1920x1080 perspective, grid + LBVH + binned k-d "
                               "(deep, MLS 32) rebuilt and rendered per TF",
                   "image": [W, H], "brick": BRICK, "step_voxels": 0.5, "path": "plain",
                   "frames": "one esk_render_multi call per step (the three structures concurrently)"},
        "phases": {
            "set_volume_ms": round(statistics.median(sv), 4),
            "set_volume_gb_per_s": {"algorithmic": round(a1_bytes / (statistics.median(sv) * 1e-3) / 1e9, 1),
                                    "algorithmic_bytes": a1_bytes,
                                    "copy_inclusive": round(sv_gbs, 1), "copy_inclusive_bytes": sv_bytes,
                                    "peak": 8000.0, "measured_copy": round(copy_gbs, 1)},
            "rebuild": {a: {k: round(v, 4) for k, v in rebuild[a].items()} for a in ACCELS},
            "render_ms": {a: round(statistics.median(render_ms[a]), 4) for a in ACCELS},
            "render_ms_in_step": {a: round(statistics.median(render_ms_step[a]), 4) for a in render_ms_step},
            "render_mrays_per_s": {a: round(W * H / statistics.median(render_ms[a]) / 1e3, 1)
                                   for a in ACCELS},
            "naive_render_ms": round(statistics.median(naive), 4),
            "naive_mrays_per_s": round(W * H / statistics.median(naive) / 1e3, 1),
            "samples_per_frame": samples,
            "gsamples_per_s": {a: round(samples[a] / (statistics.median(render_ms[a]) * 1e-3) / 1e9, 2)
                               for a in ACCELS},
            "bricks_nonempty": st["n_nonempty"], "lbvh_nodes": st["lbvh_nodes"],
            "lbvh_height": st["lbvh_height"], "kd_nodes": st["kd_nodes"], "kd_height": st["kd_height"],
            "shallow_kd_and_hybrid": shallow,
            "voxel_tight": tight,
        },
        "roofline": {"kernel": f"k_render<{dominant}>", "bound": "alu", "achieved": round(achieved, 3),
                     "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / PEAK_FP32_TFLOPS, 5), "traffic": measured_traffic(dominant),
                     "work": {"flop_per_sample": FLOP_PER_SAMPLE, "samples": sum(step_samples),
                              "launches": args.steps, "ms": round(sum(dom_ms), 4)},
                     "issue": None if issue is None else {
                         "valu_wave_instr_per_launch": issue["VALU instr"],
                         "lane_instr_per_sample": issue["lane instr / sample"],
                         "valu_issue_frac": issue["VALU issue"],
                         "peak_wave_instr_per_s": PEAK_VALU_WAVE_INSTR_PER_S,
                         "l2_requests_per_launch": issue["L2 requests"], "l2_hit": issue["L2 hit"],
                         "source": "profiles/render_issue_noise512_1080p.md"}},
    }
    log("small configuration (64^3 u8, 128x128)")
    result["small_config"] = small_config(esk, torch)
    if not args.no_batch:
        log("batched vs plain")
        result["batched"] = batched_vs_plain(esk, torch)
        log("serving")
        result["serving"] = serving(esk, torch)
        log("graph replay")
        result["graph_replay"] = graph_replay(esk, torch)
    if not args.no_stats:
        log("node/height statistics")
        result["statistics"] = statistics_table(esk, torch, dvol)
        log("sort paths (radix sort vs Morton enumeration)")
        result["sort_paths"] = sort_paths(esk, torch)
    if not args.no_large:
        log("large volumes (1024^3 f32/f16, 2048^3 u16)")
        result["large_volumes"] = large_volumes(esk, torch)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        result["cpu_baseline"] = cpu_baseline(vol, tfs, args.cpu_steps, args.cpu_stride)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
