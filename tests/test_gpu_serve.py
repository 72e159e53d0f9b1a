"""Serving with continuous batching: every result equals serving the same
requests one at a time in arrival order, bit for bit, also when the memory
budget forces requests to wait for earlier batches."""
import numpy as np
import pytest

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
    for i, dims in enumerate([(48, 40, 56), (64, 64, 32), (30, 72, 50), (96, 48, 64)]):
        vols[f"v{i}"] = (synth.blobs_u8(dims, seed=seed + i, n_blobs=5, cut=40), dims,
                         synth.tf_random(seed * 10 + i, 256))
    reqs, t = [], 0.0
    for rid in range(n_req):
        t += rng.exponential(1.0 / rate)
        name = f"v{int(rng.integers(0, 4))}"
        if rng.random() < 0.4:
            tf = torch.from_numpy(synth.tf_random(seed * 1000 + rid, 256)).cuda()
            reqs.append(Request(rid, name, "rebuild", t, tf=tf))
        else:
            W, H = int(rng.choice([48, 64, 96])), int(rng.choice([40, 64, 80]))
            cam = synth.perspective(vols[name][1], W, H, synth.view_direction(seed * 1000 + rid))
            reqs.append(Request(rid, name, "render", t, cam=cam, size=(W, H)))
    return vols, reqs


def replay_alone(vols, reqs):
    """The same requests, one at a time, in arrival order, plain calls."""
    torch = _torch()
    import paper_1912_09596_amd as esk
    ctxs = {}
    for name, (vol, dims, tf) in vols.items():
        c = esk.Context(0)
        c.set_volume(torch.from_numpy(vol).cuda(), 8, max_tf=256)
        c.set_tf(torch.from_numpy(tf).cuda(), build=("lbvh",))
        ctxs[name] = c
    out = {}
    for r in sorted(reqs, key=lambda r: (r.arrival, r.rid)):
        if r.kind == "rebuild":
            ctxs[r.volume].set_tf(r.tf, build=("lbvh",))
        else:
            out[r.rid] = ctxs[r.volume].render(r.cam, r.size[0], r.size[1], accel="lbvh").cpu().numpy()
    return out


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
    ref = replay_alone(vols, reqs)
    for r in reqs:
        if r.kind == "render":
            assert np.array_equal(r.out.cpu().numpy(), ref[r.rid]), r.rid
