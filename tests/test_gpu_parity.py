"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Integer work (min/max, flags, grid, compaction, Morton keys, sort, LBVH,
k-d tree) must match bit for bit; images must be within 1e-3 max-abs RGBA of
the FP64 oracle, per-pixel sample counts must match exactly, and every
skipping mode must reproduce the GPU's own full march bit for bit."""
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

TOL = 1e-3
# (halting, max leaf size, bins): the paper's 4 bins for every halting
# rule, and the other bin counts the ABI accepts
KD_VARIANTS = [(0, 0, 4), (1, 0, 4), (1, 32, 4), (1, 128, 4), (1, 0, 2), (0, 0, 3), (1, 32, 8), (1, 0, 16)]


def kd_bins(kd):
    return kd[2] if len(kd) > 2 else 4


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def to_dev(a):
    torch = _torch()
    if a.dtype == np.uint16:
        return torch.from_numpy(a.view(np.int16).copy()).view(torch.uint16).cuda()
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def make_ctx():
    import paper_1912_09596_amd as esk
    _torch()
    return esk, esk.Context(0)


def check_hierarchies(ctx, vol, tf, B, lo=0.0, hi=1.0, kd=(1, 0), label=""):
    """Compares every rebuild product with the oracle, bit for bit."""
    nz, ny, nx = vol.shape
    dims = (nx, ny, nz)
    mn, mx = oracle.brick_minmax(vol, B)
    gmn, gmx = ctx.export("minmax")
    assert np.array_equal(gmn.astype(np.float64), mn), label
    assert np.array_equal(gmx.astype(np.float64), mx), label
    assert np.array_equal(ctx.export("tf_prefix"), oracle.tf_prefix(tf)), label
    flags = oracle.classify(mn, mx, vol.dtype, tf, lo, hi)
    assert np.array_equal(ctx.export("flags"), flags), label
    grid = ctx.export("grid")
    bits = np.unpackbits(grid.view(np.uint8), bitorder="little")[: flags.size]
    assert np.array_equal(bits, flags), label
    ids = oracle.compact(flags)
    assert np.array_equal(ctx.export("ids"), ids), label
    nb = oracle.brick_grid(dims, B)
    keys = oracle.morton_keys(ids, nb[0], nb[1])
    assert np.array_equal(ctx.export("keys"), keys), label
    sk, si = oracle.sort_pairs(keys, ids)
    assert np.array_equal(ctx.export("sorted_keys"), sk), label
    assert np.array_equal(ctx.export("sorted_ids"), si), label
    t = oracle.lbvh(sk, si, B, dims)
    for name in ("left", "right", "axis", "lo", "hi"):
        assert np.array_equal(ctx.export("lbvh_" + name), t[name]), (label, name)
    st = ctx.stats()
    assert st["n_nonempty"] == ids.size, label
    assert st["lbvh_height"] == t["height"], label
    assert st["lbvh_nodes"] == (2 * ids.size - 1 if ids.size else 0)
    k = oracle.kd(flags, B, dims, kd[0], kd[1], kd_bins(kd))
    for name in ("lo", "hi", "axis", "plane"):
        assert np.array_equal(ctx.export("kd_" + name), k[name]), (label, name)
    assert np.array_equal(ctx.export("kd_first"), k["first_child"]), label
    assert st["kd_nodes"] == len(k["axis"]) and st["kd_height"] == k["height"], label
    return flags


def run_case(vol, tf, B, lo=0.0, hi=1.0, kd=(1, 0), label=""):
    esk, ctx = make_ctx()
    torch = _torch()
    dv = to_dev(vol)
    dtf = to_dev(tf)
    ctx.set_volume(dv, B, (lo, hi), max_tf=max(256, tf.shape[0]))
    ctx.set_tf(dtf, build=("grid", "lbvh", "kd"), kd=esk.Kd(kd[0], kd[1], kd_bins(kd)))
    torch.cuda.synchronize()
    flags = check_hierarchies(ctx, vol, tf, B, lo, hi, kd, label)
    return esk, ctx, flags, dv, dtf


def check_images(ctx, vol, tf, cam, W, H, flags, B, lo=0.0, hi=1.0, dt=0.5, ref=1.0, label=""):
    torch = _torch()
    ref_img, ref_cnt = oracle.render(vol, tf, cam, W, H, dt, ref, lo, hi, with_counts=True)
    _, skip_cnt = oracle.render(vol, tf, cam, W, H, dt, ref, lo, hi, mode=1, flags=flags, B=B,
                                with_counts=True)
    imgs = {}
    for accel in ("none", "grid", "lbvh", "kd", "hybrid"):
        cnt = torch.empty((H, W), dtype=torch.int32, device="cuda")
        img = ctx.render(cam, W, H, accel=accel, step=dt, ref=ref, counts=cnt)
        torch.cuda.synchronize()
        img, cnt = img.cpu().numpy(), cnt.cpu().numpy()
        err = np.abs(img.astype(np.float64) - ref_img).max()
        assert err <= TOL, (label, accel, err)
        if accel == "none":
            assert np.array_equal(cnt, ref_cnt), (label, "sample set differs from the oracle")
        elif accel in ("grid", "lbvh", "hybrid"):
            # exactly the samples of non-empty bricks: the grid (also inside
            # the hybrid's k-d leaves) and the LBVH, whose leaves are bricks
            assert np.array_equal(cnt, skip_cnt), (label, accel)
        else:
            assert np.all(cnt >= skip_cnt) and np.all(cnt <= ref_cnt), label
        imgs[accel] = img
    for accel in ("grid", "lbvh", "kd", "hybrid"):
        assert np.array_equal(imgs[accel], imgs["none"]), (label, accel, "skip != full march")
    return imgs


def test_c1_workload_full_parity():
    w = synth.c1_workload()
    log("case: C1 64^3 u8 blobs, B=8")
    esk, ctx, flags, _, _ = run_case(w["vol"], w["tf"], w["brick"], label="C1")
    assert 0 < flags.mean() < 1
    check_images(ctx, w["vol"], w["tf"], w["cam"], w["W"], w["H"], flags, w["brick"], label="C1")
    cam = synth.orthographic((64, 64, 64), 96, 80, synth.view_direction(5))
    check_images(ctx, w["vol"], w["tf"], cam, 96, 80, flags, w["brick"], label="C1 ortho")


@pytest.mark.parametrize("dims,B,dtype,seed", [
    ((37, 50, 29), 8, np.uint8, 0),
    ((45, 33, 52), 16, np.float32, 1),
    ((61, 40, 47), 8, np.float16, 2),
    ((70, 23, 38), 4, np.uint16, 3),
    ((100, 90, 70), 32, np.uint8, 4),
    # FP32 bricks of 8 and 32 voxels: min/max combined from the blocked
    # copy's per-block summaries (1 and 4 stored blocks per brick axis)
    ((29, 37, 23), 8, np.float32, 5),
    ((70, 41, 99), 32, np.float32, 6),
])
def test_ragged_volumes(dims, B, dtype, seed):
    log(f"case: ragged {dims} B={B} {np.dtype(dtype).name} seed={seed}")
    base = synth.blobs_u8(dims, seed=50 + seed, n_blobs=7, cut=40)
    if dtype == np.uint8:
        vol = base
    elif dtype == np.uint16:
        vol = (base.astype(np.uint16) * 257).astype(np.uint16)
    else:
        vol = (base.astype(np.float64) / 255.0).astype(dtype)
    tf = synth.tf_random(seed + 10, 256)
    for kd in KD_VARIANTS:
        esk, ctx, flags, _, _ = run_case(vol, tf, B, kd=kd, label=f"{dims} kd={kd}")
    W, H = 72, 56
    for i, ortho in enumerate((0, 1)):
        d = synth.view_direction(seed * 3 + i)
        cam = synth.orthographic(dims, W, H, d) if ortho else synth.perspective(dims, W, H, d)
        check_images(ctx, vol, tf, cam, W, H, flags, B, label=f"{dims} ortho={ortho}")


def test_far_cameras():
    # rays ending beyond t = 16384 take leaf sample ranges widened by a
    # sample on each side (FP32 error of the slab values grows with t)
    w = synth.c1_workload()
    log("case: C1 seen from ~22000 voxels (perspective and orthographic)")
    esk, ctx, flags, _, _ = run_case(w["vol"], w["tf"], w["brick"], label="far")
    cam = synth.perspective((64, 64, 64), 64, 48, synth.view_direction(7), fovy_deg=0.25, dist=200.0)
    assert float(np.linalg.norm(cam["eye"] - 32.0)) > 16384 + 200
    check_images(ctx, w["vol"], w["tf"], cam, 64, 48, flags, w["brick"], label="far perspective")
    cam = synth.orthographic((64, 64, 64), 64, 48, synth.view_direction(8), dist=200.0)
    check_images(ctx, w["vol"], w["tf"], cam, 64, 48, flags, w["brick"], label="far ortho")


def test_float_value_range_and_opacity_modes():
    log("case: f32 with value range [-2, 3], dt 0.05 / 0.37 / 1.0 / 2.3 / 7.9, ref 0 / 1 / 2")
    dims = (40, 36, 44)
    base = synth.blobs_u8(dims, seed=77, n_blobs=6, cut=30).astype(np.float64)
    vol = (base / 255.0 * 5.0 - 2.0).astype(np.float32)
    tf = synth.tf_random(99, 300)
    esk, ctx, flags, _, _ = run_case(vol, tf, 8, lo=-2.0, hi=3.0, label="range")
    cam = synth.perspective(dims, 64, 48, synth.view_direction(9))
    # fine and coarse steps (a step longer than a brick skips whole leaves)
    for dt, ref in ((0.37, 1.0), (1.0, 0.0), (0.5, 2.0), (0.05, 1.0), (2.3, 1.0), (7.9, 0.0)):
        check_images(ctx, vol, tf, cam, 64, 48, flags, 8, lo=-2.0, hi=3.0, dt=dt, ref=ref,
                     label=f"dt={dt} ref={ref}")


def test_degenerate_occupancies():
    dims = (48, 40, 56)
    vol = synth.blobs_u8(dims, seed=3, n_blobs=5, cut=50)
    cam = synth.perspective(dims, 48, 40, synth.view_direction(2))
    # all-zero alpha: nothing flagged, empty trees, black image
    tf = synth.tf_ramp(256)
    zero = tf.copy()
    zero[:, 3] = 0
    log("case: empty TF")
    esk, ctx, flags, _, _ = run_case(vol, zero, 8, label="empty TF")
    assert flags.sum() == 0
    imgs = check_images(ctx, vol, zero, cam, 48, 40, flags, 8, label="empty TF")
    assert np.all(imgs["lbvh"] == 0)
    # every entry visible: every brick flagged
    full = tf.copy()
    full[:, 3] = 0.05
    log("case: full TF")
    esk, ctx, flags, _, _ = run_case(vol, full, 8, label="full TF")
    assert flags.all()
    check_images(ctx, vol, full, cam, 48, 40, flags, 8, label="full TF")
    # exactly one and exactly two non-empty bricks
    for spots in ([(20, 20, 20)], [(3, 4, 5), (44, 36, 50)]):
        v = np.zeros(dims[::-1], np.uint8)
        for (x, y, z) in spots:
            v[z, y, x] = 250
        log(f"case: spots {spots}")
        only = np.zeros((256, 4), np.float32)
        only[200:, :] = [1.0, 0.5, 0.25, 0.9]
        esk, ctx, flags, _, _ = run_case(v, only, 32, label=f"spots {spots}")
        check_images(ctx, v, only, cam, 48, 40, flags, 32, label=f"spots {spots}")


def test_tf_alpha_out_of_range():
    """Opacities outside [0, 1] and NaN are read clamped (NaN as 0) by every
    step: hierarchies exact, images within tolerance of the oracle's and
    every skipping mode equal to the full march."""
    dims = (41, 37, 30)
    vol = synth.blobs_u8(dims, seed=12, n_blobs=6, cut=40)
    tf = synth.tf_random(21, 256)
    a = tf[:, 3].copy()
    a[40:60] = -0.3
    a[90:95] = np.nan
    a[150:170] = 1.8
    a[200:203] = np.inf
    tf[:, 3] = a
    log("case: TF alpha with negative, NaN, > 1 and inf entries")
    esk, ctx, flags, _, _ = run_case(vol, tf, 8, label="alpha clamp")
    assert 0 < flags.mean() < 1
    cam = synth.perspective(dims, 56, 48, synth.view_direction(13))
    imgs = check_images(ctx, vol, tf, cam, 56, 48, flags, 8, label="alpha clamp")
    assert np.isfinite(imgs["none"]).all()


def test_menger_sponge_kd_root_only():
    vol = synth.menger_sponge(3, 3)
    dims = vol.shape[::-1]
    tf = synth.tf_ramp(256)
    log("case: Menger sponge")
    for kd in ((0, 0), (1, 0), (1, 32)):
        esk, ctx, flags, _, _ = run_case(vol, tf, 4, kd=kd, label=f"menger {kd}")
    assert ctx.stats()["kd_nodes"] > 1
    cam = synth.perspective(dims, 64, 64, synth.view_direction(11))
    check_images(ctx, vol, tf, cam, 64, 64, flags, 4, label="menger")


def test_multiblock_sort_path():
    # more than 32768 bricks -> the multi-block radix sort
    dims = (300, 260, 200)
    log(f"case: multi-block sort {dims} B=4")
    vol = synth.blobs_u8(dims, seed=8, n_blobs=40, sigma=(6.0, 14.0), cut=20, centre_range=(0.05, 0.95))
    tf = synth.tf_ramp(256, start=0.05)
    esk, ctx, flags, _, _ = run_case(vol, tf, 4, label="multiblock")
    assert ctx.stats()["n_bricks"] > 32768 and flags.sum() > 32768


def test_kd_levels_wider_than_block_numbering():
    """Thin tubes in 320^3 voxels, 4^3 bricks (512,000 bricks): the k-d trees
    hold levels of more than 2048 nodes, whose children are numbered by the
    last workgroup of their own level launch instead of by every workgroup of
    the next one, so the build switches between both ways and back; every
    node, the first-child links and the height bit-exact against the oracle,
    and the k-d render equal to the full march."""
    torch = _torch()
    dims = (320, 320, 320)
    log(f"case: k-d wide levels {dims} B=4")
    vol = synth.tubes(dims, n_tubes=300, seed=3, radius=(1.0, 2.0))
    tf = synth.tf_ramp(256, start=0.05)
    B = 4
    esk, ctx = make_ctx()
    ctx.set_volume(to_dev(vol), B, (0.0, 1.0), max_tf=256)
    dtf = to_dev(tf)
    mn, mx = oracle.brick_minmax(vol, B)
    flags = oracle.classify(mn, mx, vol.dtype, tf)
    cam = synth.perspective(dims, 96, 64, synth.view_direction(5))
    for kd in ((1, 0), (1, 32)):
        log(f"case: k-d wide levels kd={kd}")
        k = oracle.kd(flags, B, dims, kd[0], kd[1], 4)
        # the premise: some level of the oracle's tree is wider than 2048 nodes
        axis, begin, end, widest = k["axis"], 0, 1, 0
        while begin < end:
            widest = max(widest, end - begin)
            begin, end = end, end + 2 * int((axis[begin:end] >= 0).sum())
        assert widest > 2048, widest
        ctx.set_tf(dtf, build=("kd",), kd=esk.Kd(kd[0], kd[1], 4))
        torch.cuda.synchronize()
        for name in ("lo", "hi", "axis", "plane"):
            assert np.array_equal(ctx.export("kd_" + name), k[name]), (kd, name)
        assert np.array_equal(ctx.export("kd_first"), k["first_child"]), kd
        st = ctx.stats()
        assert st["kd_nodes"] == len(k["axis"]) and st["kd_height"] == k["height"], kd
        full = ctx.render(cam, 96, 64, accel="none").cpu().numpy()
        img = ctx.render(cam, 96, 64, accel="kd").cpu().numpy()
        assert np.array_equal(img, full), kd


def test_render_multi_equals_single_renders():
    """esk_render_multi: each frame bit-identical to esk_render of the same
    request (grid, LBVH, k-d, hybrid and the full march, counts included),
    the frames of different structures running on different streams; read
    back on the context's stream with no synchronisation of our own (the call
    joins its frames), twice, with a rebuild between."""
    torch = _torch()
    dims = (96, 80, 72)
    log(f"case: render_multi {dims} B=8")
    vol = synth.blobs_u8(dims, seed=3, n_blobs=10, sigma=(4.0, 9.0), cut=40, centre_range=(0.1, 0.9))
    esk, ctx = make_ctx()
    ctx.set_volume(to_dev(vol), 8, (0.0, 1.0), max_tf=256)
    W, H = 120, 90
    for rnd, tf in enumerate((synth.tf_ramp(256, start=0.05), synth.tf_random(7, 256))):
        ctx.set_tf(to_dev(tf), build=("grid", "lbvh", "kd"), kd=esk.Kd(1, 32, 4))
        cam = synth.perspective(dims, W, H, synth.view_direction(rnd + 2))
        accels = ("grid", "lbvh", "kd", "hybrid", "none")
        frames = [dict(cam=cam, W=W, H=H, accel=a) for a in accels]
        frames[1]["counts"] = torch.zeros((H, W), dtype=torch.int32, device="cuda")
        frames[2]["counts"] = torch.zeros((H, W), dtype=torch.int32, device="cuda")
        outs = ctx.render_multi(frames)
        got = [o.cpu().numpy() for o in outs]
        got_cnt = {i: frames[i]["counts"].cpu().numpy() for i in (1, 2)}
        for i, a in enumerate(accels):
            cnt = torch.zeros((H, W), dtype=torch.int32, device="cuda")
            ref = ctx.render(cam, W, H, accel=a, counts=cnt).cpu().numpy()
            assert np.array_equal(got[i], ref), (rnd, a)
            if i in got_cnt:
                assert np.array_equal(got_cnt[i], cnt.cpu().numpy()), (rnd, a)
        assert np.array_equal(got[0], got[4]) and np.array_equal(got[1], got[4]), rnd


def test_rebuild_is_deterministic():
    w = synth.c1_workload()
    esk, ctx = make_ctx()
    torch = _torch()
    ctx.set_volume(to_dev(w["vol"]), 8, max_tf=256)
    tf = to_dev(synth.tf_random(5, 256))
    outs = []
    for _ in range(3):
        ctx.set_tf(tf, build=("grid", "lbvh", "kd"), kd=esk.Kd(1, 32, 4))
        outs.append({k: ctx.export(k) for k in ("lbvh_left", "lbvh_right", "lbvh_lo", "lbvh_hi",
                                                "kd_lo", "kd_axis", "kd_first")})
        img = ctx.render(w["cam"], 128, 128, accel="lbvh")
        torch.cuda.synchronize()
        outs[-1]["img"] = img.cpu().numpy()
    for o in outs[1:]:
        for k in o:
            assert np.array_equal(o[k], outs[0][k]), k


def test_back_to_back_rebuilds_and_renders():
    """Rebuilds of every structure and LBVH / grid / k-d renders enqueued back
    to back with no synchronisation (the LBVH and k-d builds run on internal
    streams): every image equals the one of the same TF rendered in a fresh
    context with a synchronisation after each call."""
    w = synth.c1_workload()
    esk, ctx = make_ctx()
    torch = _torch()
    vol = to_dev(w["vol"])
    ctx.set_volume(vol, 8, max_tf=256)
    tfs = [to_dev(synth.tf_random(40 + i, 256)) for i in range(6)]
    log("case: back-to-back rebuilds and renders")
    got = []
    for tf in tfs:
        ctx.set_tf(tf, build=("grid", "lbvh", "kd"), kd=esk.Kd(1, 32, 4))
        got.append([ctx.render(w["cam"], 96, 80, accel=a) for a in ("lbvh", "grid", "kd")])
    torch.cuda.synchronize()
    for i, tf in enumerate(tfs):
        _, ref = make_ctx()
        ref.set_volume(vol, 8, max_tf=256)
        ref.set_tf(tf, build=("grid", "lbvh", "kd"), kd=esk.Kd(1, 32, 4))
        ref.sync()
        for j, a in enumerate(("lbvh", "grid", "kd")):
            img = ref.render(w["cam"], 96, 80, accel=a)
            torch.cuda.synchronize()
            assert torch.equal(got[i][j], img), (i, a)
        ref.close()


def test_context_reuse_across_volumes_and_sizes():
    esk, ctx = make_ctx()
    torch = _torch()
    for dims, B in (((64, 64, 64), 8), ((33, 70, 21), 16), ((64, 64, 64), 4)):
        log(f"case: reuse {dims} B={B}")
        vol = synth.blobs_u8(dims, seed=sum(dims), n_blobs=4)
        tf = synth.tf_random(sum(dims), 256)
        ctx.set_volume(to_dev(vol), B, max_tf=256)
        ctx.set_tf(to_dev(tf), build=("grid", "lbvh", "kd"), kd=esk.Kd(1, 0, 4))
        torch.cuda.synchronize()
        check_hierarchies(ctx, vol, tf, B, label=f"reuse {dims}")


@pytest.mark.slow
def test_c2_full_size_sampled():
    """512^3 f32 noise, 16^3 bricks, 1920x1080: hierarchies exact for several
    TFs of the sequence; images on sampled pixels the oracle renders one by one."""
    torch = _torch()
    log("case: C2 512^3 f32 (generating volume)")
    vol = synth.fractal_noise((512, 512, 512), seed=2)
    tfs = synth.c2_tfs(100)
    esk, ctx = make_ctx()
    dv = to_dev(vol)
    ctx.set_volume(dv, 16, (0.0, 1.0), max_tf=256)
    rng = np.random.default_rng(0)
    W, H = 1920, 1080
    for i in (0, 1, 49, 99):
        log(f"case: C2 TF {i}")
        tf = tfs[i]
        for kd in ((0, 0), (1, 32)):
            ctx.set_tf(to_dev(tf), build=("grid", "lbvh", "kd"), kd=esk.Kd(kd[0], kd[1], 4))
            torch.cuda.synchronize()
            flags = check_hierarchies(ctx, vol, tf, 16, kd=kd, label=f"C2 tf{i} kd{kd}")
        cam = synth.c2_camera(i)
        pix = np.stack([rng.integers(0, W, 400), rng.integers(0, H, 400)], 1).astype(np.int32)
        ref_img, ref_cnt = oracle.render(vol, tf, cam, W, H, pixels=pix, with_counts=True)
        full = None
        for accel in ("none", "grid", "lbvh", "kd", "hybrid"):
            cnt = torch.empty((H, W), dtype=torch.int32, device="cuda")
            img = ctx.render(cam, W, H, accel=accel, counts=cnt).cpu().numpy()
            cnt = cnt.cpu().numpy()
            got = img[pix[:, 1], pix[:, 0]].astype(np.float64)
            assert np.abs(got - ref_img).max() <= TOL, (i, accel)
            if accel == "none":
                assert np.array_equal(cnt[pix[:, 1], pix[:, 0]], ref_cnt)
                full = img
            else:
                assert np.array_equal(img, full), (i, accel)


@pytest.mark.parametrize("dims,B,dtype,seed", [
    ((45, 38, 29), 8, np.uint8, 0),
    ((52, 33, 41), 4, np.float32, 1),
    ((70, 64, 36), 16, np.float16, 2),
])
def test_per_voxel_vote(dims, B, dtype, seed):
    """The per-voxel vote (Sec. 3.1): flags bit-exact against the oracle's
    vote, hierarchies built from them exact, and skipped renders equal to the
    oracle's render that skips the same bricks (the vote is not conservative,
    so they may differ from the full march)."""
    torch = _torch()
    log(f"case: vote {dims} B={B} {np.dtype(dtype).name}")
    base = synth.blobs_u8(dims, seed=90 + seed, n_blobs=6, cut=40)
    vol = base if dtype == np.uint8 else (base.astype(np.float64) / 255.0).astype(dtype)
    tf = synth.tf_random(seed + 40, 256)
    esk, ctx = make_ctx()
    ctx.set_volume(to_dev(vol), B, max_tf=256)
    ctx.set_tf(to_dev(tf), build=("grid", "lbvh", "kd"), kd=esk.Kd(1, 0, 4), classify="voxel")
    torch.cuda.synchronize()
    v = oracle.vote(vol, B, tf)
    assert np.array_equal(ctx.export("flags"), v)
    mn, mx = oracle.brick_minmax(vol, B)
    assert np.all(v <= oracle.classify(mn, mx, vol.dtype, tf))
    ids = oracle.compact(v)
    assert np.array_equal(ctx.export("ids"), ids)
    nb = oracle.brick_grid(dims, B)
    sk, si = oracle.sort_pairs(oracle.morton_keys(ids, nb[0], nb[1]), ids)
    t = oracle.lbvh(sk, si, B, dims)
    for name in ("left", "right", "lo", "hi"):
        assert np.array_equal(ctx.export("lbvh_" + name), t[name]), name
    k = oracle.kd(v, B, dims, 1, 0)
    for name in ("lo", "hi", "axis", "plane"):
        assert np.array_equal(ctx.export("kd_" + name), k[name]), name
    W, H = 64, 48
    cam = synth.perspective(dims, W, H, synth.view_direction(seed + 7))
    ref, ref_cnt = oracle.render(vol, tf, cam, W, H, mode=1, flags=v, B=B, with_counts=True)
    full = oracle.render(vol, tf, cam, W, H)
    for accel in ("grid", "lbvh", "kd"):
        cnt = torch.empty((H, W), dtype=torch.int32, device="cuda")
        img = ctx.render(cam, W, H, accel=accel, counts=cnt)
        torch.cuda.synchronize()
        img, cnt = img.cpu().numpy().astype(np.float64), cnt.cpu().numpy()
        assert np.abs(img - ref).max() <= TOL, accel
        if accel == "grid":
            assert np.array_equal(cnt, ref_cnt)
        else:
            assert np.all(cnt >= ref_cnt)
    log(f"  vote flags {int(v.sum())} of {v.size} bricks (min/max: "
        f"{int(oracle.classify(mn, mx, vol.dtype, tf).sum())}); max|vote render - full march| "
        f"{np.abs(ref - full).max():.2e}")


@pytest.mark.parametrize("dims,B,dtype,seed", [
    ((45, 38, 29), 8, np.uint8, 0),
    ((52, 33, 41), 4, np.float32, 1),
    ((70, 64, 36), 16, np.float16, 2),
    ((61, 40, 47), 8, np.uint16, 3),
])
def test_voxel_tight_boxes(dims, B, dtype, seed):
    """Voxel-tight boxes: the per-brick boxes bit-exact against the oracle;
    every mode still reproduces the full march bit for bit; the LBVH (leaves
    = bricks) composites exactly the samples inside their bricks' tight boxes,
    the k-d tree and the hybrid grid at least those and at most the full or
    the brick-skipping sets."""
    torch = _torch()
    log(f"case: tight boxes {dims} B={B} {np.dtype(dtype).name}")
    base = synth.blobs_u8(dims, seed=110 + seed, n_blobs=6, cut=40)
    if dtype == np.uint8:
        vol = base
    elif dtype == np.uint16:
        vol = (base.astype(np.uint16) * 257).astype(np.uint16)
    else:
        vol = (base.astype(np.float64) / 255.0).astype(dtype)
    tf = synth.tf_random(seed + 50, 256)
    esk, ctx = make_ctx()
    ctx.set_volume(to_dev(vol), B, max_tf=256)
    for kd in ((1, 0), (0, 0)):
        ctx.set_tf(to_dev(tf), build=("grid", "lbvh", "kd"), kd=esk.Kd(kd[0], kd[1], 4), tight=True)
        torch.cuda.synchronize()
        mn, mx = oracle.brick_minmax(vol, B)
        flags = oracle.classify(mn, mx, vol.dtype, tf)
        assert np.array_equal(ctx.export("flags"), flags)
        boxes = oracle.tight_boxes(vol, B, tf, flags)
        assert np.array_equal(ctx.export("tight"), boxes)
        # the exported hierarchies are those of the brick flags, unchanged
        k = oracle.kd(flags, B, dims, kd[0], kd[1])
        assert np.array_equal(ctx.export("kd_lo"), k["lo"]) and np.array_equal(ctx.export("kd_axis"), k["axis"])
        W, H = 64, 48
        cam = synth.perspective(dims, W, H, synth.view_direction(seed + 11))
        ref, _ = oracle.render(vol, tf, cam, W, H, with_counts=True)
        _, c_brick = oracle.render(vol, tf, cam, W, H, mode=1, flags=flags, B=B, with_counts=True)
        _, c_tight = oracle.render(vol, tf, cam, W, H, mode=2, flags=flags, B=B, boxes=boxes, with_counts=True)
        imgs = {}
        for accel in ("none", "grid", "lbvh", "kd", "hybrid"):
            cnt = torch.empty((H, W), dtype=torch.int32, device="cuda")
            img = ctx.render(cam, W, H, accel=accel, counts=cnt)
            torch.cuda.synchronize()
            img, cnt = img.cpu().numpy(), cnt.cpu().numpy()
            assert np.abs(img.astype(np.float64) - ref).max() <= TOL, accel
            imgs[accel] = img
            if accel == "lbvh":
                assert np.array_equal(cnt, c_tight), (kd, accel)
            elif accel == "grid":
                assert np.array_equal(cnt, c_brick), (kd, accel)
            elif accel == "hybrid":
                assert np.all(cnt >= c_tight) and np.all(cnt <= c_brick), (kd, accel)
            elif accel == "kd":
                assert np.all(cnt >= c_tight), (kd, accel)
        for accel in ("grid", "lbvh", "kd", "hybrid"):
            assert np.array_equal(imgs[accel], imgs["none"]), (kd, accel)
        log(f"  kd={kd}: samples full {int(ref.shape[0])}x, brick {int(c_brick.sum())}, tight {int(c_tight.sum())}")


def test_compaction_on_export():
    """The brick ids and their Morton keys are compacted in the rebuild only
    where a later step reads them (voxel-tight boxes, the radix sort), else
    when exported: every export must show the current classification, after
    rebuilds that compacted and rebuilds that did not, across TFs and
    volumes, and in either export order."""
    esk, ctx = make_ctx()
    torch = _torch()
    steps = [
        # (dims, B, build, tight, tf seed, export keys first)
        ((64, 64, 64), 8, ("grid",), False, 1, True),      # no compaction in the rebuild
        ((64, 64, 64), 8, ("grid",), False, 2, False),     # new TF: the old ids must not show
        ((64, 64, 64), 8, ("lbvh",), False, 3, True),      # sorted keys by enumeration
        ((64, 64, 64), 8, ("grid",), True, 4, False),      # compacted for the tight boxes
        ((64, 64, 64), 8, ("kd",), False, 5, True),
        ((200, 24, 24), 8, ("lbvh",), False, 6, False),    # 25x3x3 bricks: radix sort
        ((200, 24, 24), 8, ("grid",), False, 7, True),
    ]
    last = None
    for dims, B, build, tight, seed, keys_first in steps:
        log(f"case: compaction on export {dims} B={B} {build} tight={tight} tf={seed}")
        vol = synth.blobs_u8(dims, seed=sum(dims), n_blobs=5, cut=40)
        tf = synth.tf_random(seed + 60, 256)
        if (dims, B) != last:
            ctx.set_volume(to_dev(vol), B, max_tf=256)
            last = (dims, B)
        ctx.set_tf(to_dev(tf), build=build, kd=esk.Kd(1, 0, 4), tight=tight)
        torch.cuda.synchronize()
        mn, mx = oracle.brick_minmax(vol, B)
        flags = oracle.classify(mn, mx, vol.dtype, tf)
        ids = oracle.compact(flags)
        nb = oracle.brick_grid(dims, B)
        keys = oracle.morton_keys(ids, nb[0], nb[1])
        order = ("keys", "ids") if keys_first else ("ids", "keys")
        got = {k: ctx.export(k) for k in order}
        assert np.array_equal(ctx.export("flags"), flags)
        assert np.array_equal(got["ids"], ids), (dims, build, seed)
        assert np.array_equal(got["keys"], keys), (dims, build, seed)
        if "lbvh" in build:
            sk, si = oracle.sort_pairs(keys, ids)
            assert np.array_equal(ctx.export("sorted_keys"), sk)
            assert np.array_equal(ctx.export("sorted_ids"), si)


@pytest.mark.parametrize("dims,B,dtype,seed", [
    ((64, 64, 64), 8, np.uint8, 0), ((61, 47, 53), 4, np.uint16, 1), ((96, 80, 72), 16, np.float32, 2),
    ((130, 66, 40), 8, np.float16, 3),
])
def test_kd_tight_split_cost(dims, B, dtype, seed):
    """The k-d build with the voxel-tight split cost (Sec. 3.2.2): every node
    bit-exact against the oracle's build from its own tight boxes, for
    shallow, deep and MLS trees and 4 or 8 bins; it differs from the
    brick-cost tree somewhere in the set; every mode still reproduces the
    full march bit for bit."""
    torch = _torch()
    log(f"case: k-d tight cost {dims} B={B} {np.dtype(dtype).name}")
    base = synth.blobs_u8(dims, seed=140 + seed, n_blobs=7, cut=30)
    if dtype == np.uint8:
        vol = base
    elif dtype == np.uint16:
        vol = (base.astype(np.uint16) * 257).astype(np.uint16)
    else:
        vol = (base.astype(np.float64) / 255.0).astype(dtype)
    tf = synth.tf_random(seed + 90, 256)
    esk, ctx = make_ctx()
    ctx.set_volume(to_dev(vol), B, max_tf=256)
    mn, mx = oracle.brick_minmax(vol, B)
    flags = oracle.classify(mn, mx, vol.dtype, tf)
    boxes = oracle.tight_boxes(vol, B, tf, flags)
    W, H = 64, 48
    cam = synth.perspective(dims, W, H, synth.view_direction(seed + 21))
    differs = False
    for halting, mls, bins in ((1, 0, 4), (0, 0, 4), (1, 16, 4), (1, 0, 8)):
        ctx.set_tf(to_dev(tf), build=("grid", "lbvh", "kd"), kd=esk.Kd(halting, mls, bins), kd_cost="tight")
        torch.cuda.synchronize()
        assert np.array_equal(ctx.export("tight"), boxes)
        k = oracle.kd(flags, B, dims, halting, mls, bins, tight_boxes=boxes)
        kb = oracle.kd(flags, B, dims, halting, mls, bins)
        differs = differs or len(k["axis"]) != len(kb["axis"]) or not np.array_equal(k["plane"], kb["plane"])
        for name in ("lo", "hi", "axis", "plane"):
            assert np.array_equal(ctx.export("kd_" + name), k[name]), (halting, mls, bins, name)
        st = ctx.stats()
        assert st["kd_nodes"] == len(k["axis"]) and st["kd_height"] == k["height"]
        full = ctx.render(cam, W, H, accel="none").cpu().numpy()
        for accel in ("kd", "hybrid"):
            img = ctx.render(cam, W, H, accel=accel).cpu().numpy()
            assert np.array_equal(img, full), (halting, mls, bins, accel)
        log(f"  halting={halting} mls={mls} bins={bins}: tight-cost nodes {len(k['axis'])} (height "
            f"{k['height']}), brick-cost nodes {len(kb['axis'])} (height {kb['height']})")
    ref = oracle.render(vol, tf, cam, W, H)
    assert np.abs(full.astype(np.float64) - ref).max() <= TOL
    assert differs
