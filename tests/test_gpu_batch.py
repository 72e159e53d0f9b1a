"""Batched rendering: many contexts (own volume, TF, hierarchy, camera and
image size) in one launch.  Every image must equal the one rendered alone,
bit for bit, and match the FP64 oracle within 1e-3."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def make_requests(count, seed):
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(count):
        dims = tuple(int(v) for v in rng.choice([24, 40, 64, 96], size=3))
        vol = synth.blobs_u8(dims, n_blobs=int(rng.integers(2, 7)), seed=seed * 100 + i, cut=40)
        tf = synth.tf_random(seed * 100 + i, 256)
        W, H = int(rng.choice([48, 64, 80])), int(rng.choice([40, 64, 72]))
        cam = synth.perspective(dims, W, H, synth.view_direction(seed * 100 + i))
        B = int(rng.choice([4, 8, 16]))
        reqs.append(dict(dims=dims, vol=vol, tf=tf, W=W, H=H, cam=cam, B=B))
    return reqs


@pytest.mark.parametrize("accel", ["lbvh", "grid", "kd", "hybrid", "none"])
def test_batched_equals_alone(accel):
    torch = _torch()
    import paper_1912_09596_amd as esk
    reqs = make_requests(12, 3)
    print(f"case: batch of {len(reqs)} requests, accel {accel}", flush=True)
    ctxs = []
    for r in reqs:
        c = esk.Context(0)
        c.set_volume(torch.from_numpy(r["vol"]).cuda(), r["B"], max_tf=256)
        c.set_tf(torch.from_numpy(r["tf"]).cuda(), build=("grid", "lbvh", "kd"), kd=esk.Kd(1, 32, 4))
        ctxs.append(c)
    alone = [c.render(r["cam"], r["W"], r["H"], accel=accel).clone() for c, r in zip(ctxs, reqs)]
    batched = esk.render_batch(ctxs, [r["cam"] for r in reqs], [(r["W"], r["H"]) for r in reqs], accel=accel)
    torch.cuda.synchronize()
    for i, (a, b) in enumerate(zip(alone, batched)):
        assert np.array_equal(a.cpu().numpy(), b.cpu().numpy()), i
    for i in (0, 5):
        r = reqs[i]
        ref = oracle.render(r["vol"], r["tf"], r["cam"], r["W"], r["H"])
        assert np.abs(batched[i].cpu().numpy().astype(np.float64) - ref).max() <= 1e-3
    # a batch of one is the plain call
    one = esk.render_batch(ctxs[:1], [reqs[0]["cam"]], [(reqs[0]["W"], reqs[0]["H"])], accel=accel)
    torch.cuda.synchronize()
    assert np.array_equal(one[0].cpu().numpy(), alone[0].cpu().numpy())


def test_brick_autotuner_choice_renders_the_same_image():
    """The autotuner measures every candidate brick size and returns the
    cheapest; the image does not depend on the brick size (every mode equals
    the full march), so a render with the chosen size equals one with any
    other size bit for bit."""
    torch = _torch()
    import paper_1912_09596_amd as esk
    from paper_1912_09596_amd.tune import tune_brick
    r = make_requests(1, 9)[0]
    vol = torch.from_numpy(r["vol"]).cuda()
    tf = torch.from_numpy(r["tf"]).cuda()
    best, res = tune_brick(vol, tf, r["cam"], (r["W"], r["H"]), accel="lbvh", reps=2)
    print(f"case: autotune {r['dims']}: {res}", flush=True)
    assert best in res and set(res) <= {8, 16, 32}
    assert res[best]["cost_ms"] == min(v["cost_ms"] for v in res.values())
    imgs = []
    for B in sorted(res):
        c = esk.Context(0)
        c.set_volume(vol, B, max_tf=256)
        c.set_tf(tf, build=("lbvh",))
        imgs.append(c.render(r["cam"], r["W"], r["H"], accel="lbvh").cpu().numpy())
        c.close()
    for im in imgs[1:]:
        assert np.array_equal(im, imgs[0])


def test_rebuild_render_graph_replays():
    """Rebuild + render captured once and replayed with three different TFs:
    every replay equals the eager rebuild + render of the same TF bit for bit
    (eager work and synchronisations between the replays), and the flags,
    brick ids and Morton keys exported after each replay are the oracle's
    for that TF (the ids and keys are made at export when the captured
    rebuild does not make them)."""
    torch = _torch()
    import paper_1912_09596_amd as esk
    from paper_1912_09596_amd.graphs import RebuildRenderGraph
    r = make_requests(1, 5)[0]
    vol = torch.from_numpy(r["vol"]).cuda()
    print(f"case: graph capture {r['dims']} {r['W']}x{r['H']}", flush=True)
    for accel in ("lbvh", "grid"):
        g = RebuildRenderGraph(vol, r["B"], 256, r["cam"], (r["W"], r["H"]), accel=accel)
        eager = esk.Context(0)
        eager.set_volume(vol, r["B"], max_tf=256)
        for seed in (11, 12, 13):
            tf = torch.from_numpy(synth.tf_random(seed, 256)).cuda()
            img = g.replay(tf)
            g.stream.synchronize()
            got = img.cpu().numpy().copy()
            eager.set_tf(tf, build=(accel,))
            want = eager.render(r["cam"], r["W"], r["H"], accel=accel).cpu().numpy()
            torch.cuda.synchronize()
            assert np.array_equal(got, want), (accel, seed)
            assert np.abs(got).max() > 0
            mn, mx = oracle.brick_minmax(r["vol"], r["B"])
            flags = oracle.classify(mn, mx, r["vol"].dtype, synth.tf_random(seed, 256))
            ids = oracle.compact(flags)
            nb = oracle.brick_grid(r["dims"], r["B"])
            assert np.array_equal(g.ctx.export("flags"), flags), (accel, seed)
            assert np.array_equal(g.ctx.export("ids"), ids), (accel, seed)
            assert np.array_equal(g.ctx.export("keys"), oracle.morton_keys(ids, nb[0], nb[1])), (accel, seed)
        eager.close()
        g.close()


def test_batched_rebuild_equals_alone():
    """All requests set their TFs and rebuild in one launch chain: the flags,
    the sorted keys and the LBVH of every context, and every image rendered
    from them, equal rebuilding each context alone, bit for bit; two images
    match the FP64 oracle within 1e-3.  The mix holds grids whose keys come
    from the Morton enumeration and lopsided ones that take the radix sort
    alone (and in the batch, the largest); a second round with new TFs
    reuses the argument buffer."""
    torch = _torch()
    import paper_1912_09596_amd as esk
    reqs = make_requests(10, 21)
    # lopsided brick grids: alone they take the radix sort (code domain above
    # 4x the brick count); in the batch the first two take the Morton
    # enumeration (domain <= 2^20 codes) and the third the radix sort too
    for i, dims in enumerate([(200, 24, 24), (24, 176, 16), (2048, 8, 8)]):
        vol = synth.blobs_u8(dims, n_blobs=4, seed=700 + i, cut=40)
        cam = synth.perspective(dims, 64, 48, synth.view_direction(700 + i))
        reqs.append(dict(dims=dims, vol=vol, tf=synth.tf_random(700 + i, 256), W=64, H=48, cam=cam, B=4))
    print(f"case: batched rebuild of {len(reqs)} requests", flush=True)
    batch, alone = [], []
    for r in reqs:
        for group in (batch, alone):
            c = esk.Context(0)
            c.set_volume(torch.from_numpy(r["vol"]).cuda(), r["B"], max_tf=256)
            group.append(c)
    args = None
    for rnd in range(2):
        tfs = [torch.from_numpy(r["tf"] if rnd == 0 else synth.tf_random(900 + i, 256)).cuda()
               for i, r in enumerate(reqs)]
        args = esk.rebuild_batch(batch, tfs, build=("grid", "lbvh"), args_buffer=args)
        imgs = esk.render_batch(batch, [r["cam"] for r in reqs], [(r["W"], r["H"]) for r in reqs], accel="lbvh")
        torch.cuda.synchronize()
        for i, (c, r) in enumerate(zip(alone, reqs)):
            c.set_tf(tfs[i], build=("grid", "lbvh"))
            want = c.render(r["cam"], r["W"], r["H"], accel="lbvh").cpu().numpy()
            assert np.array_equal(imgs[i].cpu().numpy(), want), (rnd, i)
            grid = c.render(r["cam"], r["W"], r["H"], accel="grid").cpu().numpy()
            got_grid = batch[i].render(r["cam"], r["W"], r["H"], accel="grid").cpu().numpy()
            assert np.array_equal(got_grid, grid), (rnd, i)
            for what in ("flags", "grid", "sorted_keys", "sorted_ids", "lbvh_left", "lbvh_right", "lbvh_axis",
                         "lbvh_lo", "lbvh_hi"):
                assert np.array_equal(batch[i].export(what), c.export(what)), (rnd, i, what)
            assert batch[i].stats() == c.stats(), (rnd, i)
        for i in (0, len(reqs) - 1):
            r = reqs[i]
            tf_np = tfs[i].cpu().numpy()
            ref = oracle.render(r["vol"], tf_np, r["cam"], r["W"], r["H"])
            assert np.abs(imgs[i].cpu().numpy().astype(np.float64) - ref).max() <= 1e-3, (rnd, i)
    for c in batch + alone:
        c.close()


def test_batched_rebuild_render_graph_replays():
    """The batched rebuild + render captured into one graph and replayed with
    three TF sets (eager work and synchronisations between the replays):
    every image equals rebuilding and rendering its request alone."""
    torch = _torch()
    import paper_1912_09596_amd as esk
    from paper_1912_09596_amd.graphs import BatchRebuildRenderGraph
    reqs = make_requests(6, 31)
    vols = [torch.from_numpy(r["vol"]).cuda() for r in reqs]
    print(f"case: batched graph of {len(reqs)} requests", flush=True)
    g = BatchRebuildRenderGraph(vols, [r["B"] for r in reqs], 256, [r["cam"] for r in reqs],
                                [(r["W"], r["H"]) for r in reqs], accel="lbvh")
    alone = []
    for r, v in zip(reqs, vols):
        c = esk.Context(0)
        c.set_volume(v, r["B"], max_tf=256)
        alone.append(c)
    for rnd in range(3):
        tfs = [torch.from_numpy(synth.tf_random(1300 + 10 * rnd + i, 256)).cuda() for i in range(len(reqs))]
        outs = g.replay(torch.stack(tfs))
        g.stream.synchronize()
        got = [o.cpu().numpy().copy() for o in outs]
        for i, (c, r) in enumerate(zip(alone, reqs)):
            c.set_tf(tfs[i], build=("lbvh",))
            want = c.render(r["cam"], r["W"], r["H"], accel="lbvh").cpu().numpy()
            torch.cuda.synchronize()
            assert np.array_equal(got[i], want), (rnd, i)
    g.close()
    for c in alone:
        c.close()
