"""The allocation-free batched render (esk_render_batch_noalloc), called
through the C ABI: its images must equal those of esk_render_batch bit for
bit, on two calls in a row, the second with fewer and smaller requests (the
static argument array keeps the first call's arguments past the second's)."""
import ctypes

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _requests(count, seed, sizes):
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(count):
        dims = tuple(int(v) for v in rng.choice([24, 40, 64], size=3))
        vol = synth.blobs_u8(dims, n_blobs=int(rng.integers(2, 6)), seed=seed * 100 + i, cut=40)
        tf = synth.tf_random(seed * 100 + i, 256)
        W, H = (int(v) for v in rng.choice(sizes, size=2))
        cam = synth.perspective(dims, W, H, synth.view_direction(seed * 100 + i))
        reqs.append(dict(vol=vol, tf=tf, W=W, H=H, cam=cam, B=int(rng.choice([4, 8, 16]))))
    return reqs


def _noalloc(L, esk, ctxs, reqs, outs, accel):
    n = len(reqs)
    ctx_arr = (ctypes.c_void_p * n)(*[c._ctx.value for c in ctxs])
    cam_arr = (esk.Camera * n)(*[esk.camera_struct(r["cam"]) for r in reqs])
    w_arr = (ctypes.c_int * n)(*[r["W"] for r in reqs])
    h_arr = (ctypes.c_int * n)(*[r["H"] for r in reqs])
    out_arr = (ctypes.c_void_p * n)(*[o.data_ptr() for o in outs])
    return L.esk_render_batch_noalloc(ctx_arr, n, esk.ACCEL[accel], cam_arr, w_arr, h_arr, 0.5, 1.0, out_arr)


@pytest.mark.parametrize("accel", ["lbvh", "kd"])
def test_noalloc_batch_equals_batch(accel):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1912_09596_amd as esk
    L = esk.lib()
    first = _requests(9, 41, [64, 80, 96])
    second = _requests(4, 42, [24, 40])
    ctxs = []
    for r in first:
        c = esk.Context(0)
        c.set_volume(torch.from_numpy(r["vol"]).cuda(), r["B"], max_tf=256)
        c.set_tf(torch.from_numpy(r["tf"]).cuda(), build=("grid", "lbvh", "kd"), kd=esk.Kd(1, 32, 4))
        ctxs.append(c)
    for call, reqs in enumerate((first, second)):
        print(f"case: no-alloc batch call {call}, {len(reqs)} requests, accel {accel}", flush=True)
        use = ctxs[:len(reqs)]
        if call == 1:
            # new volumes, TFs and cameras for the smaller second call
            for c, r in zip(use, reqs):
                c.set_volume(torch.from_numpy(r["vol"]).cuda(), r["B"], max_tf=256)
                c.set_tf(torch.from_numpy(r["tf"]).cuda(), build=("grid", "lbvh", "kd"), kd=esk.Kd(1, 32, 4))
        ref = esk.render_batch(use, [r["cam"] for r in reqs], [(r["W"], r["H"]) for r in reqs], accel=accel)
        outs = [torch.full((r["H"], r["W"], 4), float("nan"), dtype=torch.float32, device="cuda") for r in reqs]
        st = _noalloc(L, esk, use, reqs, outs, accel)
        assert st == esk.OK, L.esk_last_error(use[0]._ctx).decode()
        torch.cuda.synchronize()
        for i, (a, b) in enumerate(zip(ref, outs)):
            assert np.array_equal(a.cpu().numpy(), b.cpu().numpy()), (call, i)
    for c in ctxs:
        c.close()
