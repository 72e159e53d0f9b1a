"""Serving with continuous batching: every result equals serving the same
requests one at a time in arrival order, bit for bit, also when the memory
budget forces requests to wait for earlier batches; and every served image
matches the FP64 oracle (the TF in effect at its arrival) within 1e-3 on
sampled pixels, for u8 and f16 volumes alike."""
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


def workload(seed, n_req=48, rate=4000.0):
    torch = _torch()
    from paper_1912_09596_amd.serve import Request
    rng = np.random.default_rng(seed)
    vols = {}
    dims_list = [(48, 40, 56), (64, 64, 32), (30, 72, 50), (96, 48, 64), (40, 56, 44), (72, 40, 40)]
    for i, dims in enumerate(dims_list):
        v = synth.blobs_u8(dims, seed=seed + i, n_blobs=5, cut=40)
        if i >= 4:
            v = (v.astype(np.float32) / 255.0).astype(np.float16)   # f16 storage, values in [0, 1]
        vols[f"v{i}"] = (v, dims, synth.tf_random(seed * 10 + i, 256))
    reqs, t = [], 0.0
    for rid in range(n_req):
        t += rng.exponential(1.0 / rate)
        name = f"v{int(rng.integers(0, len(vols)))}"
        if rng.random() < 0.4:
            tf_np = synth.tf_random(seed * 1000 + rid, 256)
            r = Request(rid, name, "rebuild", t, tf=torch.from_numpy(tf_np).cuda())
            r.tf_np = tf_np
            reqs.append(r)
        else:
            W, H = int(rng.choice([48, 64, 96])), int(rng.choice([40, 64, 80]))
            cam = synth.perspective(vols[name][1], W, H, synth.view_direction(seed * 1000 + rid))
            reqs.append(Request(rid, name, "render", t, cam=cam, size=(W, H)))
    return vols, reqs


def replay_alone(vols, reqs):
    """The same requests, one at a time, in arrival order, plain calls; also
    the TF in effect for every render."""
    torch = _torch()
    import paper_1912_09596_amd as esk
    ctxs, cur = {}, {}
    for name, (vol, dims, tf) in vols.items():
        c = esk.Context(0)
        c.set_volume(torch.from_numpy(vol).cuda(), 8, max_tf=256)
        c.set_tf(torch.from_numpy(tf).cuda(), build=("lbvh",))
        ctxs[name] = c
        cur[name] = tf
    out, tf_at = {}, {}
    for r in sorted(reqs, key=lambda r: (r.arrival, r.rid)):
        if r.kind == "rebuild":
            ctxs[r.volume].set_tf(r.tf, build=("lbvh",))
            cur[r.volume] = r.tf_np
        else:
            out[r.rid] = ctxs[r.volume].render(r.cam, r.size[0], r.size[1], accel="lbvh").cpu().numpy()
            tf_at[r.rid] = cur[r.volume]
    return out, tf_at


@pytest.mark.parametrize("tight_budget", [False, True])
def test_serving_matches_one_at_a_time(tight_budget):
    torch = _torch()
    from paper_1912_09596_amd.serve import Server
    vols, reqs = workload(11)
    srv = Server(hbm_budget_bytes=1 << 40, max_batch=16)
    for name, (vol, dims, tf) in vols.items():
        srv.add_volume(name, torch.from_numpy(vol).cuda(), 8, tf=torch.from_numpy(tf).cuda())
    if tight_budget:
        # room for the resident volumes plus about two output images
        srv.budget = srv.resident + 2 * 96 * 80 * 16
    print(f"case: serving {len(reqs)} requests, tight budget {tight_budget}", flush=True)
    stats = srv.run(reqs)
    torch.cuda.synchronize()
    assert all(r.done is not None and r.done >= r.arrival for r in reqs)
    assert stats["p50_ms"] is not None and stats["p99_ms"] >= stats["p50_ms"]
    ref, tf_at = replay_alone(vols, reqs)
    rng = np.random.default_rng(5)
    worst = 0.0
    for r in reqs:
        if r.kind != "render":
            continue
        got = r.out.cpu().numpy()
        assert np.array_equal(got, ref[r.rid]), r.rid
        # the FP64 oracle on sampled pixels, with the TF in effect at arrival
        W, H = r.size
        pix = np.stack([rng.integers(0, W, 24), rng.integers(0, H, 24)], 1).astype(np.int32)
        exp = oracle.render(vols[r.volume][0], tf_at[r.rid], r.cam, W, H, pixels=pix)
        err = float(np.abs(got[pix[:, 1], pix[:, 0]].astype(np.float64) - exp).max())
        worst = max(worst, err)
        assert err <= 1e-3, (r.rid, r.volume, err)
    print(f"served renders vs FP64 oracle (sampled pixels): max |err| = {worst:.2e}", flush=True)
