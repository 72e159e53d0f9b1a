"""Pins of the CPU oracle against facts other than itself: closed forms,
invariants, brute force on tiny inputs, an independent construction
algorithm, and the paper's printed table.  No GPU needed."""
import math
import os

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------------------
# a1: brick min/max with a one-voxel apron
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("dims,B", [((16, 16, 16), 8), ((37, 50, 29), 8), ((33, 17, 40), 16)])
def test_minmax_constant_volume(dims, B):
    nx, ny, nz = dims
    vol = np.full((nz, ny, nx), 77, np.uint8)
    mn, mx = oracle.brick_minmax(vol, B)
    nb = np.prod(oracle.brick_grid(dims, B))
    assert mn.shape == (nb,) and np.all(mn == 77) and np.all(mx == 77)


@pytest.mark.parametrize("dims,B", [((37, 5, 6), 8), ((64, 3, 3), 16), ((41, 9, 9), 32)])
def test_minmax_ramp_closed_form(dims, B):
    # v = x: the apron of brick bx spans x in [B*bx - 1, B*bx + B] clipped,
    # so min = max(0, B*bx - 1) and max = min(nx - 1, B*bx + B).
    nx, ny, nz = dims
    vol = np.broadcast_to(np.arange(nx, dtype=np.uint16)[None, None, :], (nz, ny, nx)).copy()
    mn, mx = oracle.brick_minmax(vol, B)
    nbx, nby, nbz = oracle.brick_grid(dims, B)
    mn = mn.reshape(nbz, nby, nbx)
    mx = mx.reshape(nbz, nby, nbx)
    for bx in range(nbx):
        assert np.all(mn[:, :, bx] == max(0, B * bx - 1))
        assert np.all(mx[:, :, bx] == min(nx - 1, B * bx + B))


@pytest.mark.parametrize("q", [(0, 0, 0), (7, 8, 3), (15, 16, 31), (8, 7, 9), (39, 39, 39)])
def test_minmax_single_spike(q):
    # A voxel on the face of a brick also lies in the face neighbour's apron.
    B, n = 8, 40
    vol = np.zeros((n, n, n), np.uint8)
    vol[q[2], q[1], q[0]] = 9
    mn, mx = oracle.brick_minmax(vol, B)
    nb = oracle.brick_grid((n, n, n), B)
    expect = np.zeros(nb[::-1], bool)
    owners = []
    for a in range(3):
        s = {q[a] // B}
        if q[a] % B == B - 1 and (q[a] + 1) // B < nb[a]:
            s.add((q[a] + 1) // B)
        if q[a] % B == 0 and q[a] > 0:
            s.add((q[a] - 1) // B)
        owners.append(s)
    for bx in owners[0]:
        for by in owners[1]:
            for bz in owners[2]:
                expect[bz, by, bx] = True
    assert np.array_equal(mx.reshape(nb[::-1]) > 0, expect)
    assert np.all(mn == 0)


def test_minmax_f16_matches_numpy_decoding():
    rng = np.random.default_rng(5)
    bits = rng.integers(0, 0x7C00, size=(9, 10, 11)).astype(np.uint16)  # finite, non-negative
    bits[0, 0, :4] = [0x0001, 0x03FF, 0x0400, 0x3C00]                   # subnormals, 1.0
    bits[1, 1, :3] |= 0x8000                                            # negatives
    vol = bits.view(np.float16)
    mn, mx = oracle.brick_minmax(vol, 8)
    ref = vol.astype(np.float64)
    assert mn.min() == ref.min() and mx.max() == ref.max()
    # brick (0,0,0) apron = voxels [0,8] on every axis (clipped to the volume)
    sub = ref[:9, :9, :9]
    assert mn[0] == sub.min() and mx[0] == sub.max()


# ---------------------------------------------------------------------------
# a2, a3: TF prefix count and classification
# ---------------------------------------------------------------------------

def test_tf_prefix_ramp_closed_form():
    # ramp TF: alpha_i > 0 iff i/255 >= 0.3, i.e. i >= 77 (76/255 < 0.3 < 77/255)
    tf = synth.tf_ramp(256, start=0.3)
    P = oracle.tf_prefix(tf)
    assert P[0] == 0 and P[-1] == 256 - 77
    for i in range(257):
        assert P[i] == max(0, i - 77)


def test_tf_alpha_read_clamped():
    # an opacity outside [0, 1] is read clamped, NaN as 0: the prefix count
    # sees NaN and -0.5 as invisible and 1.7 as visible
    tf = np.zeros((5, 4), np.float32)
    tf[:, 3] = [np.nan, -0.5, 1.7, 0.0, 0.3]
    assert list(oracle.tf_prefix(tf)) == [0, 0, 0, 1, 1, 2]
    # constant volume, every entry with alpha 1.7: the first sample is opaque
    # (1 - (1 - 1)^(dt/ref) = 1), so every hit pixel is exactly (rgb, 1)
    nx, ny, nz = 8, 6, 10
    vol = np.full((nz, ny, nx), 90, np.uint8)
    cam = _axis_camera(nx, ny)
    tf = np.zeros((256, 4), np.float32)
    tf[:] = [0.25, 0.5, 0.75, 1.7]
    img = oracle.render(vol, tf, cam, nx, ny, dt=0.5, ref=1.0)
    assert np.all(img == np.array([0.25, 0.5, 0.75, 1.0]))
    # negative or NaN opacity everywhere: nothing is visible
    for bad in (-0.5, np.nan):
        tf[:, 3] = bad
        assert np.all(oracle.render(vol, tf, cam, nx, ny) == 0.0)
        assert np.all(oracle.sample(vol, tf, [[2.5, 2.5, 2.5]])[:, 3] == 0.0)


def test_classify_tf_extremes():
    vol = synth.blobs_u8((40, 24, 33), seed=4)
    mn, mx = oracle.brick_minmax(vol, 8)
    tf = synth.tf_ramp(256)
    zero = tf.copy()
    zero[:, 3] = 0
    assert oracle.classify(mn, mx, vol.dtype, zero).sum() == 0
    full = tf.copy()
    full[:, 3] = 0.25
    assert np.all(oracle.classify(mn, mx, vol.dtype, full) == 1)


@pytest.mark.parametrize("entry,flagged", [(98, 0), (99, 1), (100, 1), (101, 1), (102, 1), (103, 0)])
def test_classify_u8_index_window(entry, flagged):
    # u8, N = 256: x(v) = v exactly, so a constant-100 brick's window is
    # [floor(x) - 1, floor(x) + 2] = [99, 102]
    vol = np.full((16, 16, 16), 100, np.uint8)
    mn, mx = oracle.brick_minmax(vol, 8)
    tf = np.zeros((256, 4), np.float32)
    tf[entry, 3] = 0.5
    assert np.all(oracle.classify(mn, mx, vol.dtype, tf) == flagged)


def test_classify_spike_between_voxel_values():
    # voxels alternate 0 / 200 along x; only entry 100 is visible.  Every voxel
    # on its own is invisible, yet the sample halfway between two voxels has
    # value 100 and is visible: the brick must be flagged.
    vol = np.zeros((16, 16, 16), np.uint8)
    vol[:, :, 1::2] = 200
    tf = np.zeros((256, 4), np.float32)
    tf[100, 3] = 0.5
    assert np.all(oracle.sample(vol, tf, [[1.5, 4.5, 4.5], [2.5, 4.5, 4.5]])[:, 3] == 0)
    mid = oracle.sample(vol, tf, [[2.0, 4.5, 4.5]])
    assert mid[0, 3] == pytest.approx(0.5)
    mn, mx = oracle.brick_minmax(vol, 8)
    assert np.all(oracle.classify(mn, mx, vol.dtype, tf) == 1)


def test_vote_spike_between_voxel_values():
    # the per-voxel vote (Sec. 3.1) looks at voxel values only: with voxels
    # alternating 0 / 200 and only entry 100 visible, no voxel votes, so the
    # vote skips a brick whose interpolated samples are visible -- the reason
    # the default classification uses min/max with an index window instead
    vol = np.zeros((16, 16, 16), np.uint8)
    vol[:, :, 1::2] = 200
    tf = np.zeros((256, 4), np.float32)
    tf[100] = (1.0, 1.0, 1.0, 0.5)
    v = oracle.vote(vol, 8, tf)
    mn, mx = oracle.brick_minmax(vol, 8)
    assert v.sum() == 0 and np.all(oracle.classify(mn, mx, vol.dtype, tf) == 1)
    cam = synth.orthographic((16, 16, 16), 12, 10, (0.3, 0.4, 1.0))
    full = oracle.render(vol, tf, cam, 12, 10)
    skipped = oracle.render(vol, tf, cam, 12, 10, mode=1, flags=v, B=8)
    assert full[..., 3].max() > 0.1 and np.all(skipped == 0)


def test_vote_tf_extremes():
    vol = synth.blobs_u8((30, 20, 25), seed=4, cut=60)
    zero = np.zeros((256, 4), np.float32)
    assert oracle.vote(vol, 8, zero).sum() == 0
    full = np.full((256, 4), 0.5, np.float32)
    assert np.all(oracle.vote(vol, 8, full) == 1)


def test_vote_single_voxel_owns_its_brick_only():
    # one bright voxel at the corner of brick (1,1,1): the vote flags exactly
    # that brick; the min/max classification (one-voxel apron) also flags the
    # seven bricks whose apron reaches the voxel
    vol = np.zeros((24, 24, 24), np.uint8)
    vol[8, 8, 8] = 255
    tf = np.zeros((256, 4), np.float32)
    tf[200:, 3] = 1.0
    v = oracle.vote(vol, 8, tf).reshape(3, 3, 3)
    expect = np.zeros((3, 3, 3), np.uint8)
    expect[1, 1, 1] = 1
    assert np.array_equal(v, expect)
    mn, mx = oracle.brick_minmax(vol, 8)
    c = oracle.classify(mn, mx, vol.dtype, tf).reshape(3, 3, 3)
    expect[0:2, 0:2, 0:2] = 1
    assert np.array_equal(c, expect)


@pytest.mark.parametrize("seed", [0, 1])
@pytest.mark.parametrize("B", [4, 8])
def test_vote_plateau_tf_closed_form(seed, B):
    # alpha 0 below entry 128, 0.5 from 128 on; voxel values avoid the band
    # 121..134 around the step, where the FP32 lookup could round either way:
    # then a brick votes iff one of its own voxels is >= 135
    rng = np.random.default_rng(seed)
    dims = (37, 29, 22)
    vals = np.concatenate([np.arange(0, 121), np.arange(135, 256)]).astype(np.uint8)
    vol = rng.choice(vals, size=dims[::-1], p=None)
    vol[rng.random(dims[::-1]) < 0.97] = 0
    tf = np.zeros((256, 4), np.float32)
    tf[128:, 3] = 0.5
    nb = oracle.brick_grid(dims, B)
    expect = np.zeros(nb[::-1], np.uint8)
    zz, yy, xx = np.nonzero(vol >= 135)
    expect[zz // B, yy // B, xx // B] = 1
    v = oracle.vote(vol, B, tf)
    assert np.array_equal(v, expect.reshape(-1))
    mn, mx = oracle.brick_minmax(vol, B)
    assert np.all(v <= oracle.classify(mn, mx, vol.dtype, tf))


@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("dtype", [np.uint8, np.uint16, np.float16, np.float32])
def test_vote_is_subset_of_classification(seed, dtype):
    # a visible voxel reads TF entries inside its brick's index window
    dims = (33, 26, 19)
    base = synth.blobs_u8(dims, seed=30 + seed, cut=40)
    if dtype == np.uint8:
        vol = base
    elif dtype == np.uint16:
        vol = (base.astype(np.uint16) * 257).astype(np.uint16)
    else:
        vol = (base.astype(np.float64) / 255.0).astype(dtype)
    tf = synth.tf_random(seed + 3, 256)
    mn, mx = oracle.brick_minmax(vol, 8)
    c = oracle.classify(mn, mx, vol.dtype, tf)
    v = oracle.vote(vol, 8, tf)
    assert v.sum() > 0 and np.all(v <= c)


def test_tight_boxes_single_voxel_closed_form():
    # one bright voxel at x = 8 (first voxel of brick 1 along x, B = 8), y = 12,
    # z = 3: the cells that read it are c = v - 1 and c = v per axis, whose
    # regions cover [v - 1/2, v + 3/2); each brick gets that range clipped to
    # itself, in half-voxel units [2v - 1, 2v + 3)
    vol = np.zeros((16, 24, 24), np.uint8)            # (z, y, x)
    vol[3, 12, 8] = 255
    tf = np.zeros((256, 4), np.float32)
    tf[128:, 3] = 1.0
    mn, mx = oracle.brick_minmax(vol, 8)
    fl = oracle.classify(mn, mx, vol.dtype, tf)
    bx = oracle.tight_boxes(vol, 8, tf, fl).reshape(2, 3, 3, 6)   # (bz, by, bx)
    assert np.array_equal(bx[0, 1, 1], [16, 23, 5, 19, 27, 9])
    assert np.array_equal(bx[0, 1, 0], [15, 23, 5, 16, 27, 9])
    # every other brick is empty (flagged or not)
    nonzero = {tuple(i) for i in np.argwhere(np.any(bx != 0, axis=-1))}
    assert nonzero == {(0, 1, 1), (0, 1, 0)}


@pytest.mark.parametrize("v", [7, 8])
def test_tight_boxes_voxel_on_brick_corner(v):
    # a bright voxel at (v, v, v) next to the corner shared by 8 bricks (B = 8):
    # the cells reading it, c in {v-1, v} per axis, cover [v - 1/2, v + 3/2),
    # and each brick gets that cube clipped to itself.  With v = 7 brick
    # (1,1,1) holds only cell (7,7,7), of which the voxel is the first corner;
    # with v = 8 brick (0,0,0) holds only cell (7,7,7), of which it is the last
    vol = np.zeros((16, 16, 16), np.uint8)
    vol[v, v, v] = 255
    tf = np.zeros((256, 4), np.float32)
    tf[128:, 3] = 1.0
    mn, mx = oracle.brick_minmax(vol, 8)
    fl = oracle.classify(mn, mx, vol.dtype, tf)
    bx = oracle.tight_boxes(vol, 8, tf, fl)
    for b in range(8):
        c = (b & 1, (b >> 1) & 1, b >> 2)
        lo = [max(2 * v - 1, 16 * c[a]) for a in range(3)]
        hi = [min(2 * v + 3, 16 * c[a] + 16) for a in range(3)]
        assert list(bx[b]) == lo + hi, (b, bx[b])


@pytest.mark.parametrize("entry,visible", [(97, False), (98, True), (99, True), (101, True), (102, False)])
def test_tight_boxes_cell_index_window(entry, visible):
    # constant u8 value 99 (x = 99 exactly for N = 256): a cell's window has
    # the brick test's margins, [99 - 1, 99 + 2], so entries 98..101 light it
    vol = np.full((12, 12, 12), 99, np.uint8)
    tf = np.zeros((256, 4), np.float32)
    tf[entry, 3] = 1.0
    fl = np.ones(8, np.uint8)
    bx = oracle.tight_boxes(vol, 8, tf, fl)
    assert np.any(bx != 0) == visible


def test_tight_boxes_full_tf_are_brick_boxes():
    dims = (27, 20, 13)
    vol = synth.blobs_u8(dims, seed=6, cut=0)
    tf = np.full((256, 4), 0.5, np.float32)
    mn, mx = oracle.brick_minmax(vol, 8)
    fl = oracle.classify(mn, mx, vol.dtype, tf)
    assert np.all(fl == 1)
    bx = oracle.tight_boxes(vol, 8, tf, fl)
    nb = oracle.brick_grid(dims, 8)
    for b in range(fl.size):
        c = (b % nb[0], (b // nb[0]) % nb[1], b // (nb[0] * nb[1]))
        lo = [2 * 8 * c[a] for a in range(3)]
        hi = [2 * min(8 * c[a] + 8, dims[a]) for a in range(3)]
        assert list(bx[b]) == lo + hi, b


@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("dtype", [np.uint8, np.float32, np.float16])
def test_tight_boxes_conservative_dense_sampling(seed, dtype):
    # every sample point with alpha > 0 lies inside its brick's tight box,
    # and every tight box lies inside its brick
    dims = (29, 23, 26)
    B = 8
    base = synth.blobs_u8(dims, seed=60 + seed, cut=40)
    vol = base if dtype == np.uint8 else (base.astype(np.float64) / 255.0).astype(dtype)
    tf = synth.tf_random(seed + 20, 256)
    mn, mx = oracle.brick_minmax(vol, B)
    fl = oracle.classify(mn, mx, vol.dtype, tf)
    bx = oracle.tight_boxes(vol, B, tf, fl)
    nb = oracle.brick_grid(dims, B)
    rng = np.random.default_rng(seed)
    pts = (rng.random((60000, 3)) * np.array(dims)).astype(np.float32)
    alpha = oracle.sample(vol, tf, pts)[:, 3]
    bid = (np.floor(pts).astype(np.int64) // B)
    lin = bid[:, 0] + nb[0] * (bid[:, 1] + nb[1] * bid[:, 2])
    box = bx[lin]
    inside = np.all((pts >= box[:, :3] * 0.5) & (pts < box[:, 3:] * 0.5), axis=1)
    assert np.all(inside[alpha > 0])
    assert inside[alpha > 0].size > 100 and (~inside).sum() > 100
    for b in np.flatnonzero(np.any(bx != 0, axis=1)):
        c = (b % nb[0], (b // nb[0]) % nb[1], b // (nb[0] * nb[1]))
        for a in range(3):
            assert 2 * B * c[a] <= bx[b, a] < bx[b, 3 + a] <= 2 * min(B * c[a] + B, dims[a])


@pytest.mark.parametrize("seed", [0, 1])
def test_render_tight_boxes_equal_full_march(seed):
    dims = (33, 28, 25)
    vol = synth.blobs_u8(dims, seed=70 + seed, n_blobs=5, cut=45)
    tf = synth.tf_random(seed + 30, 256)
    mn, mx = oracle.brick_minmax(vol, 8)
    fl = oracle.classify(mn, mx, vol.dtype, tf)
    bx = oracle.tight_boxes(vol, 8, tf, fl)
    cam = synth.perspective(dims, 40, 30, synth.view_direction(seed + 3))
    full, c0 = oracle.render(vol, tf, cam, 40, 30, with_counts=True)
    brick, c1 = oracle.render(vol, tf, cam, 40, 30, mode=1, flags=fl, B=8, with_counts=True)
    tight, c2 = oracle.render(vol, tf, cam, 40, 30, mode=2, flags=fl, B=8, boxes=bx, with_counts=True)
    assert np.array_equal(full, tight) and np.array_equal(full, brick)
    assert np.all(c2 <= c1) and np.all(c1 <= c0) and c2.sum() < c1.sum()


@pytest.mark.parametrize("entry,flagged", [(2, 0), (3, 1), (4, 1), (6, 1), (7, 0)])
def test_classify_u16_index_window_exact(entry, flagged):
    # u16, N = 256: x(v) = v * 255 / 65535 = v / 257, so the constant value
    # 1028 sits exactly on entry 4 and the window is [4 - 1, 4 + 2] = [3, 6].
    # (A single-precision 1028 * (1/65535) * 255 rounds to 3.9999998, which
    # would shift the window to [2, 5].)
    vol = np.full((12, 12, 12), 1028, np.uint16)
    mn, mx = oracle.brick_minmax(vol, 8)
    tf = np.zeros((256, 4), np.float32)
    tf[entry, 3] = 0.5
    assert np.all(oracle.classify(mn, mx, vol.dtype, tf) == flagged)


@pytest.mark.parametrize("N,entry,flagged", [(256, 114, 0), (256, 115, 1), (256, 118, 1), (256, 119, 0),
                                             (1000, 455, 0), (1000, 456, 1), (1000, 459, 1), (1000, 460, 0)])
def test_classify_u16_index_window_fraction(N, entry, flagged):
    # u16 value 30000: x = 30000 * 255 / 65535 = 116.73 (window [115, 118]);
    # with N = 1000, x = 30000 * 999 / 65535 = 457.31 (window [456, 459])
    vol = np.full((10, 9, 11), 30000, np.uint16)
    mn, mx = oracle.brick_minmax(vol, 8)
    tf = np.zeros((N, 4), np.float32)
    tf[entry, 3] = 0.25
    assert np.all(oracle.classify(mn, mx, vol.dtype, tf) == flagged)


@pytest.mark.parametrize("dtype", [np.float32, np.float16])
@pytest.mark.parametrize("value,visible", [
    (0.5, {126: 1, 129: 1, 125: 0, 130: 0}),     # s = (0.5 + 2) / 5 = 0.5, x = 127.5: window [126, 129]
    (3.7, {254: 1, 255: 1, 253: 0}),             # above hi: s = 1, x = 255: window [254, 255]
    (-2.5, {0: 1, 2: 1, 3: 0}),                  # below lo: s = 0, x = 0: window [0, 2]
    (-1.0, {50: 1, 53: 1, 49: 0, 54: 0}),        # s = 0.2, x = 51 (0.2f * 255 rounds to 51): window [50, 53]
])
def test_classify_float_value_range(dtype, value, visible):
    # f16/f32 volumes are normalised by s = clamp((v - lo) / (hi - lo), 0, 1)
    # with the value range [lo, hi] = [-2, 3]: dividing by hi instead of
    # hi - lo, or adding lo, moves every window above
    vol = np.full((9, 10, 11), value, dtype)
    mn, mx = oracle.brick_minmax(vol, 8)
    for entry, flagged in visible.items():
        tf = np.zeros((256, 4), np.float32)
        tf[entry, 3] = 0.5
        got = oracle.classify(mn, mx, vol.dtype, tf, -2.0, 3.0)
        assert np.all(got == flagged), (value, entry)


@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("dtype,vrange", [(np.uint8, None), (np.uint16, None), (np.float32, (0.0, 1.0)),
                                          (np.float16, (0.0, 1.0)), (np.float32, (-2.0, 3.0)),
                                          (np.float16, (-2.0, 3.0))])
def test_classify_conservative_dense_sampling(seed, dtype, vrange):
    # every sample point owned by an unflagged brick must have alpha exactly 0
    dims = (35, 27, 30)
    B = 8
    base = synth.blobs_u8(dims, seed=10 + seed, cut=40)
    lo, hi = vrange if vrange else (0.0, 1.0)
    if dtype == np.uint8:
        vol = base
    elif dtype == np.uint16:
        # spread over the whole u16 range, with values between the multiples of 257
        vol = (base.astype(np.uint32) * 257 + (base.astype(np.uint32) * 97) % 257).clip(0, 65535).astype(np.uint16)
    elif lo == 0.0:
        vol = (base.astype(np.float64) / 255.0).astype(dtype)
    else:
        # [-2.5, 3.5]: values below lo and above hi clamp to the TF's ends
        vol = (base.astype(np.float64) / 255.0 * 6.0 - 2.5).astype(dtype)
    tf = synth.tf_random(seed, 256)
    mn, mx = oracle.brick_minmax(vol, B)
    flags = oracle.classify(mn, mx, vol.dtype, tf, lo, hi)
    nb = oracle.brick_grid(dims, B)
    rng = np.random.default_rng(seed)
    empty = np.flatnonzero(flags == 0)
    assert 0 < empty.size < flags.size
    for b in empty[:: max(1, empty.size // 40)]:
        bx, by, bz = b % nb[0], (b // nb[0]) % nb[1], b // (nb[0] * nb[1])
        lo3 = np.array([bx, by, bz]) * B
        hi3 = np.minimum(lo3 + B, dims)
        pts = rng.uniform(lo3, hi3, size=(400, 3)).astype(np.float32)
        corners = np.array([[lo3[0], lo3[1], lo3[2]],
                            [np.nextafter(np.float32(hi3[0]), 0), lo3[1], lo3[2]],
                            [lo3[0], np.nextafter(np.float32(hi3[1]), 0), np.nextafter(np.float32(hi3[2]), 0)]],
                           np.float32)
        pts = np.concatenate([pts, corners])
        pts = np.minimum(pts, np.nextafter(hi3.astype(np.float32), 0))
        a = oracle.sample(vol, tf, pts, lo, hi)[:, 3]
        assert np.all(a == 0.0), (b, a.max())


# ---------------------------------------------------------------------------
# a4 - a6: compaction, Morton codes, sort
# ---------------------------------------------------------------------------

def test_compact_matches_nonzero():
    rng = np.random.default_rng(3)
    flags = (rng.random(5000) < 0.2).astype(np.uint8)
    ids = oracle.compact(flags)
    assert np.all(np.diff(ids.astype(np.int64)) > 0)
    assert np.array_equal(ids, np.flatnonzero(flags).astype(np.uint32))
    assert oracle.compact(np.zeros(10, np.uint8)).size == 0


def test_morton_vectors():
    assert oracle.morton3(1, 0, 0) == 4
    assert oracle.morton3(0, 1, 0) == 2
    assert oracle.morton3(0, 0, 1) == 1
    assert oracle.morton3(1023, 1023, 1023) == 2 ** 30 - 1
    assert oracle.morton3(3, 0, 0) == 4 | 32
    assert oracle.morton3(0, 2, 5) == (1 << 0) | (1 << 4) | (1 << 6)
    # z-order inside a 2x2x2 cell
    for x in (0, 1):
        for y in (0, 1):
            for z in (0, 1):
                assert oracle.morton3(x, y, z) == 4 * x + 2 * y + z


def _decode(code):
    x = y = z = 0
    for i in range(10):
        x |= ((code >> (3 * i + 2)) & 1) << i
        y |= ((code >> (3 * i + 1)) & 1) << i
        z |= ((code >> (3 * i)) & 1) << i
    return x, y, z


def test_morton_round_trip_and_keys():
    rng = np.random.default_rng(1)
    for _ in range(300):
        x, y, z = (int(v) for v in rng.integers(0, 1024, 3))
        assert _decode(oracle.morton3(x, y, z)) == (x, y, z)
    nbx, nby = 13, 7
    ids = np.array([0, 5, 13, 91, 13 * 7 * 3 + 4], np.uint32)
    keys = oracle.morton_keys(ids, nbx, nby)
    for i, k in zip(ids, keys):
        assert _decode(int(k)) == (int(i) % nbx, (int(i) // nbx) % nby, int(i) // (nbx * nby))


def test_sort_pairs_is_sorted_permutation():
    rng = np.random.default_rng(2)
    ids = np.sort(rng.choice(32 ** 3, 3000, replace=False)).astype(np.uint32)
    keys = oracle.morton_keys(ids, 32, 32)
    k, i = oracle.sort_pairs(keys, ids)
    assert np.all(np.diff(k.astype(np.int64)) > 0)
    assert np.array_equal(np.sort(i), ids)
    assert np.array_equal(oracle.morton_keys(i, 32, 32), k)


# ---------------------------------------------------------------------------
# a7, a8: LBVH against Karras's per-node construction (independent algorithm)
# ---------------------------------------------------------------------------

def _clz32(v):
    return 32 - int(v).bit_length()


def karras_per_node(keys):
    """Karras (2012), one internal node at a time: direction from the
    neighbours' common prefixes, range end by doubling + binary search,
    split by binary search.  Written independently of the oracle's
    top-down recursion."""
    n = len(keys)
    keys = [int(k) for k in keys]

    def delta(i, j):
        if j < 0 or j >= n:
            return -1
        return _clz32(keys[i] ^ keys[j])

    left, right = [], []
    for i in range(n - 1):
        d = 1 if delta(i, i + 1) - delta(i, i - 1) > 0 else -1
        dmin = delta(i, i - d)
        lmax = 2
        while delta(i, i + lmax * d) > dmin:
            lmax *= 2
        l, t = 0, lmax // 2
        while t >= 1:
            if delta(i, i + (l + t) * d) > dmin:
                l += t
            t //= 2
        j = i + l * d
        dnode = delta(i, j)
        s, div = 0, 2
        while True:
            t = -(-l // div)
            if delta(i, i + (s + t) * d) > dnode:
                s += t
            if t == 1:
                break
            div *= 2
        g = i + s * d + min(d, 0)
        left.append((oracle.LEAF | g) if min(i, j) == g else g)
        right.append((oracle.LEAF | (g + 1)) if max(i, j) == g + 1 else g + 1)
    return np.array(left, np.uint32), np.array(right, np.uint32)


def _brick_boxes(ids, B, dims):
    nb = oracle.brick_grid(dims, B)
    ids = np.asarray(ids, np.int64)
    c = np.stack([ids % nb[0], (ids // nb[0]) % nb[1], ids // (nb[0] * nb[1])], 1)
    lo = c * B
    hi = np.minimum(lo + B, np.array(dims))
    return lo, hi


@pytest.mark.parametrize("seed,dims,B", [(0, (64, 64, 64), 8), (1, (37, 50, 29), 8),
                                         (2, (100, 60, 80), 16), (3, (64, 64, 64), 32)])
def test_lbvh_matches_karras_and_brute_force(seed, dims, B):
    vol = synth.blobs_u8(dims, seed=20 + seed, n_blobs=8)
    mn, mx = oracle.brick_minmax(vol, B)
    flags = oracle.classify(mn, mx, vol.dtype, synth.tf_ramp(256, start=0.25))
    ids = oracle.compact(flags)
    nb = oracle.brick_grid(dims, B)
    k, i = oracle.sort_pairs(oracle.morton_keys(ids, nb[0], nb[1]), ids)
    t = oracle.lbvh(k, i, B, dims)
    n = len(k)
    assert n >= 2
    L, R = karras_per_node(k)
    assert np.array_equal(t["left"], L) and np.array_equal(t["right"], R)
    # every internal node is a child exactly once (except the root), every leaf exactly once
    kids = np.concatenate([L, R])
    inner = kids[(kids & oracle.LEAF) == 0]
    leaves = kids[(kids & oracle.LEAF) != 0] & ~np.uint32(oracle.LEAF)
    assert sorted(inner.tolist()) == list(range(1, n - 1))
    assert sorted(leaves.tolist()) == list(range(n))
    # leaves are exactly the flagged bricks (the spec coverage invariant)
    assert np.array_equal(np.sort(t["ids"]), np.flatnonzero(flags).astype(np.uint32))
    blo, bhi = _brick_boxes(t["ids"], B, dims)

    def walk(node, depth):
        if node & oracle.LEAF:
            j = int(node & ~np.uint32(oracle.LEAF))
            return [j], depth
        a, da = walk(int(L[node]), depth + 1)
        b, db = walk(int(R[node]), depth + 1)
        cover = a + b
        assert sorted(cover) == list(range(min(cover), max(cover) + 1))  # contiguous range
        assert np.array_equal(t["lo"][node], blo[cover].min(0))
        assert np.array_equal(t["hi"][node], bhi[cover].max(0))
        hb = (int(k[min(cover)]) ^ int(k[max(cover)])).bit_length() - 1
        assert t["axis"][node] == 2 - hb % 3
        return cover, max(da, db)

    cover, depth = walk(0, 1)
    assert sorted(cover) == list(range(n))
    assert t["height"] == depth
    # children sit on the two sides of the split plane along the split axis
    for node in range(n - 1):
        a = t["axis"][node]
        lc, rc = int(L[node]), int(R[node])
        lhi = bhi[lc & 0x7FFFFFFF][a] if lc & oracle.LEAF else t["hi"][lc][a]
        rlo = blo[rc & 0x7FFFFFFF][a] if rc & oracle.LEAF else t["lo"][rc][a]
        assert lhi <= rlo


def test_lbvh_small_cases():
    # 1 brick: a single leaf, height 1; 2 bricks: 3 nodes, height 2
    t = oracle.lbvh(np.array([5], np.uint32), np.array([3], np.uint32), 8, (32, 32, 32))
    assert t["height"] == 1 and t["left"].size == 0
    t = oracle.lbvh(np.array([0, 7], np.uint32), np.array([0, 21], np.uint32), 8, (32, 32, 32))
    assert t["height"] == 2
    assert t["left"][0] == oracle.LEAF | 0 and t["right"][0] == oracle.LEAF | 1
    assert oracle.lbvh(np.zeros(0, np.uint32), np.zeros(0, np.uint32), 8, (8, 8, 8))["height"] == 0


# ---------------------------------------------------------------------------
# a10: k-d tree
# ---------------------------------------------------------------------------

class PrefixCount:
    """3-D inclusive prefix count over brick flags with O(1) box counts, and
    tight boxes by binary search on counts -- a second way to find the
    tight boxes the oracle finds by scanning."""

    def __init__(self, flags, nb):
        f = flags.reshape(nb[2], nb[1], nb[0]).astype(np.int64)
        S = np.zeros((nb[2] + 1, nb[1] + 1, nb[0] + 1), np.int64)
        S[1:, 1:, 1:] = f.cumsum(0).cumsum(1).cumsum(2)
        self.S = S

    def count(self, lo, hi):
        S = self.S
        x0, y0, z0 = lo
        x1, y1, z1 = hi
        if x1 <= x0 or y1 <= y0 or z1 <= z0:
            return 0
        return int(S[z1, y1, x1] - S[z0, y1, x1] - S[z1, y0, x1] - S[z1, y1, x0]
                   + S[z0, y0, x1] + S[z0, y1, x0] + S[z1, y0, x0] - S[z0, y0, x0])

    def tight(self, lo, hi):
        if self.count(lo, hi) == 0:
            return None
        tlo, thi = list(lo), list(hi)
        for a in range(3):
            a0, a1 = lo[a], hi[a] - 1          # smallest c with count([lo, c]) > 0
            while a0 < a1:
                m = (a0 + a1) // 2
                h = list(hi)
                h[a] = m + 1
                if self.count(lo, h) > 0:
                    a1 = m
                else:
                    a0 = m + 1
            tlo[a] = a0
            b0, b1 = lo[a], hi[a] - 1          # largest c with count([c, hi)) > 0
            while b0 < b1:
                m = (b0 + b1 + 1) // 2
                l = list(lo)
                l[a] = m
                if self.count(l, hi) > 0:
                    b0 = m
                else:
                    b1 = m - 1
            thi[a] = b0 + 1
        return tlo, thi


def _vol(lo, hi, B, dims):
    return int(np.prod([min(B * hi[a], dims[a]) - B * lo[a] for a in range(3)]))


def check_kd(t, flags, B, dims, halting, max_leaf, bins=4):
    nb = oracle.brick_grid(dims, B)
    pc = PrefixCount(flags, nb)
    m = len(t["axis"])
    if flags.sum() == 0:
        assert m == 0
        return
    assert m % 2 == 1                                    # full binary: 2L - 1 nodes
    assert list(t["lo"][0]) == pc.tight((0, 0, 0), nb)[0]
    assert list(t["hi"][0]) == pc.tight((0, 0, 0), nb)[1]
    vroot = _vol(t["lo"][0], t["hi"][0], B, dims)
    parents = np.full(m, -1)
    depth = np.ones(m, int)
    cover = np.zeros(nb[::-1], int)
    for i in range(m):
        lo, hi = [int(v) for v in t["lo"][i]], [int(v) for v in t["hi"][i]]
        V = _vol(lo, hi, B, dims)
        allowed = (10 * V > vroot) if halting == 0 else (V > 512)
        cands = []
        if allowed:
            for a in range(3):
                e = hi[a] - lo[a]
                if e < 2:
                    continue
                planes = sorted({lo[a] + (j * e) // bins for j in range(1, bins)} - {lo[a], hi[a]})
                for p in planes:
                    l1 = list(hi)
                    l1[a] = p
                    r0 = list(lo)
                    r0[a] = p
                    TL, TR = pc.tight(lo, l1), pc.tight(r0, hi)
                    cost = _vol(*TL, B, dims) + _vol(*TR, B, dims)
                    cands.append((cost, a, p))
        best = min(cands) if cands else None            # ties: lower axis, then lower plane
        if t["axis"][i] < 0:
            assert t["first_child"][i] == -1
            assert best is None or best[0] >= V
            if best is not None and max_leaf > 0:
                assert V <= max_leaf ** 3
            cover[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] += 1
            continue
        a, p, c = int(t["axis"][i]), int(t["plane"][i]), int(t["first_child"][i])
        assert best is not None
        if best[0] < V:
            assert (a, p) == (best[1], best[2])
        else:                                           # forced middle split (max leaf size)
            assert max_leaf > 0 and V > max_leaf ** 3
            ext = [min(B * hi[q], dims[q]) - B * lo[q] if hi[q] - lo[q] >= 2 else -1 for q in range(3)]
            assert a == int(np.argmax(ext)) and p == lo[a] + (hi[a] - lo[a]) // 2
        assert c > i and c + 1 < m
        for side, child in ((0, c), (1, c + 1)):
            assert parents[child] == -1
            parents[child] = i
            depth[child] = depth[i] + 1
            rlo, rhi = list(lo), list(hi)
            if side == 0:
                rhi[a] = p
            else:
                rlo[a] = p
            tl, th = pc.tight(rlo, rhi)
            assert list(t["lo"][child]) == tl and list(t["hi"][child]) == th
    assert np.all(parents[1:] >= 0)
    assert t["height"] == depth.max()
    f3 = flags.reshape(nb[::-1]).astype(bool)
    assert np.all(cover <= 1)                           # leaves are disjoint
    assert np.all(cover[f3] == 1)                       # and cover every non-empty brick
    # BFS order: depth never decreases with the node index
    assert np.all(np.diff(depth) >= 0)


@pytest.mark.parametrize("bins", [2, 3, 4, 8, 16])
@pytest.mark.parametrize("halting,max_leaf", [(0, 0), (1, 0), (1, 32), (1, 128)])
@pytest.mark.parametrize("seed,dims,B", [(0, (64, 64, 64), 8), (1, (50, 37, 61), 8), (2, (96, 96, 64), 16)])
def test_kd_rules(seed, dims, B, halting, max_leaf, bins):
    vol = synth.blobs_u8(dims, seed=30 + seed, n_blobs=7)
    mn, mx = oracle.brick_minmax(vol, B)
    flags = oracle.classify(mn, mx, vol.dtype, synth.tf_ramp(256, start=0.3))
    t = oracle.kd(flags, B, dims, halting, max_leaf, bins)
    check_kd(t, flags, B, dims, halting, max_leaf, bins)


@pytest.mark.parametrize("bins,split", [(2, False), (3, False), (4, False), (8, True), (16, True)])
def test_kd_bins_closed_form(bins, split):
    # 16 x 2 x 2 bricks, all non-empty except the slab x = 2.  Only a plane at
    # x = 2 or 3 separates the two solid parts (cost 8 + 52 brick volumes
    # against the root's 64); every other plane, on any axis, costs exactly
    # the root's volume.  Candidate planes on the x axis are lo + floor(j*16/bins):
    # bins 2 -> {8}, 3 -> {5, 10}, 4 -> {4, 8, 12}: no split; bins 8 -> {2, 4, ...}
    # and 16 -> {1, 2, 3, ...}: split at 2 (the smaller plane of the tie 2 / 3)
    f = np.ones((2, 2, 16), np.uint8)       # [z][y][x]
    f[:, :, 2] = 0
    t = oracle.kd(f.reshape(-1), 8, (128, 16, 16), 1, 0, bins)
    if not split:
        assert len(t["axis"]) == 1 and t["axis"][0] == -1
        return
    assert len(t["axis"]) == 3 and t["height"] == 2
    assert t["axis"][0] == 0 and t["plane"][0] == 2 and t["first_child"][0] == 1
    assert list(t["lo"][1]) == [0, 0, 0] and list(t["hi"][1]) == [2, 2, 2]
    assert list(t["lo"][2]) == [3, 0, 0] and list(t["hi"][2]) == [16, 2, 2]


def test_kd_menger_root_only():
    # empty space enclosed by the volume: the greedy cost never improves on the
    # root, so shallow and deep (no MLS) trees are a single node of height 1,
    # as printed for the Menger sponge in the statistics table.
    vol = synth.menger_sponge(3, 3)
    dims = vol.shape[::-1]
    mn, mx = oracle.brick_minmax(vol, 3)
    flags = oracle.classify(mn, mx, vol.dtype, synth.tf_ramp(256, start=0.3))
    assert 0 < flags.mean() < 1
    for halting in (0, 1):
        t = oracle.kd(flags, 3, dims, halting, 0)
        assert len(t["axis"]) == 1 and t["height"] == 1
    t = oracle.kd(flags, 3, dims, 1, 32)
    check_kd(t, flags, 3, dims, 1, 32)
    assert len(t["axis"]) > 1


def test_kd_solid_and_forced_octants():
    flags = np.ones(8 ** 3, np.uint8)      # solid 64^3 voxels in 8^3 bricks
    dims = (64, 64, 64)
    for halting in (0, 1):
        t = oracle.kd(flags, 8, dims, halting, 0)
        assert len(t["axis"]) == 1 and t["height"] == 1
    # MLS 32: split at the middle of the largest extent until every leaf is 32^3
    t = oracle.kd(flags, 8, dims, 1, 32)
    assert len(t["axis"]) == 15 and t["height"] == 4
    leaves = sorted(tuple(t["lo"][i]) for i in range(15) if t["axis"][i] < 0)
    assert leaves == sorted((x, y, z) for x in (0, 4) for y in (0, 4) for z in (0, 4))
    assert list(t["axis"][:3]) == [0, 1, 1]


def test_kd_two_blobs_first_split_separates():
    nb = 16
    f = np.zeros((nb, nb, nb), np.uint8)
    f[5:9, 6:10, 0:2] = 1      # [z][y][x]: blob at x in [0,2)
    f[5:9, 6:10, 14:16] = 1    # blob at x in [14,16)
    t = oracle.kd(f.reshape(-1), 8, (128, 128, 128), 1, 0)
    # planes at 4, 8, 12 all separate the blobs at equal cost: the smallest wins
    assert t["axis"][0] == 0 and t["plane"][0] == 4
    assert list(t["lo"][1]) == [0, 6, 5] and list(t["hi"][1]) == [2, 10, 9]
    assert list(t["lo"][2]) == [14, 6, 5] and list(t["hi"][2]) == [16, 10, 9]


def test_table_statistics_reading():
    """The statistics table: every tree is full binary (odd node counts, one
    entry marked suspect), a single node has height 1, three nodes height 2."""
    rows = [l.split() for l in open(os.path.join(GOLDEN, "table_statistics.txt"))
            if l.strip() and not l.startswith("#")]
    suspect = {("NBody1024", 0)}
    for r in rows:
        vals = [int(v) for v in r[1:]]
        for c in range(7):
            nodes, height = vals[2 * c], vals[2 * c + 1]
            if (r[0], c) not in suspect:
                assert nodes % 2 == 1, (r[0], c)
            if nodes == 1:
                assert height == 1
            if nodes == 3:
                assert height == 2
            assert nodes <= 2 ** height - 1
    # our trees follow the same reading
    t = oracle.kd(np.ones(1, np.uint8), 8, (8, 8, 8), 1, 0)
    assert len(t["axis"]) == 1 and t["height"] == 1
    f = np.zeros(8, np.uint8)
    f[[0, 7]] = 1
    t = oracle.kd(f, 8, (16, 16, 16), 1, 0)
    assert len(t["axis"]) == 3 and t["height"] == 2


# ---------------------------------------------------------------------------
# a11 - a14: the image
# ---------------------------------------------------------------------------

def _axis_camera(nx, ny):
    # orthographic, looking along +z from z = -1; pixel (x, y) -> ray through
    # voxel column (x + .5, ny - y - .5)
    return dict(ortho=1, eye=np.array([0, ny, -1], np.float32),
                dir00=np.array([0, 0, 1], np.float32),
                du=np.array([1, 0, 0], np.float32), dv=np.array([0, -1, 0], np.float32))


def test_render_constant_volume_closed_form():
    nx, ny, nz = 12, 10, 16
    vol = np.full((nz, ny, nx), 128, np.uint8)
    tf = np.zeros((256, 4), np.float32)
    tf[:] = [0.2, 0.5, 0.7, 0.3]
    img, cnt = oracle.render(vol, tf, _axis_camera(nx, ny), nx, ny, dt=0.5, ref=1.0, with_counts=True)
    assert np.all(cnt == 2 * nz)                         # K = (t_exit - t_entry) / dt samples
    A = 1.0 - (1.0 - np.float64(np.float32(0.3))) ** nz  # (1 - a')^K = (1 - a)^(K dt)
    assert np.allclose(img[..., 3], A, rtol=0, atol=1e-12)
    rgb = np.array([np.float32(0.2), np.float32(0.5), np.float32(0.7)], np.float64)
    assert np.allclose(img[..., :3], rgb * A, rtol=0, atol=1e-12)
    # no opacity correction: ref = 0 equals ref = dt = 1
    i0 = oracle.render(vol, tf, _axis_camera(nx, ny), nx, ny, dt=1.0, ref=0.0)
    i1 = oracle.render(vol, tf, _axis_camera(nx, ny), nx, ny, dt=1.0, ref=1.0)
    assert np.allclose(i0, i1, rtol=0, atol=1e-15)


@pytest.mark.parametrize("dt", [0.5, 0.3, 1.0])
def test_render_linear_ramp_closed_form(dt):
    # v = z, s = v / (nz - 1), alpha = kappa * s (a linear TF is exact under
    # the TF lerp), cell-centred trilinear reproduces v(p) = clamp(p_z - 1/2).
    nx, ny, nz = 6, 5, 20
    vol = np.broadcast_to(np.arange(nz, dtype=np.float32)[:, None, None], (nz, ny, nx)).copy()
    N, kappa = 64, 0.1
    tf = np.zeros((N, 4), np.float32)
    tf[:, 0] = 1.0
    tf[:, 3] = (kappa * np.arange(N) / (N - 1)).astype(np.float32)
    img = oracle.render(vol, tf, _axis_camera(nx, ny), nx, ny, dt=dt, ref=1.0, lo=0.0, hi=nz - 1.0)
    trans = 1.0
    k = 0
    while True:
        t = np.float32(1.0) + np.float32(np.float32(k) + np.float32(0.5)) * np.float32(dt)
        if not t < np.float32(1 + nz):
            break
        pz = np.float32(-1.0) + t
        s = min(max(float(pz) - 0.5, 0.0), nz - 1.0) / (nz - 1.0)
        trans *= (1.0 - kappa * s) ** (np.float32(dt) / 1.0)
        k += 1
    A = 1.0 - trans
    assert np.allclose(img[..., 3], A, rtol=0, atol=2e-7)   # TF entries are float32
    assert np.allclose(img[..., 0], A, rtol=0, atol=2e-7)


def test_render_orientation_and_empty_tf():
    dims = (32, 32, 32)
    vol = np.zeros((32, 32, 32), np.uint8)
    vol[20:28, 20:28, 20:28] = 200         # x, y, z all in the upper half
    tf = synth.tf_ramp(256)
    cam = synth.perspective(dims, 64, 64, direction=(0.0, 0.0, 1.0))
    img = oracle.render(vol, tf, cam, 64, 64)
    A = img[..., 3]
    assert A.max() > 0.5
    assert np.all(A[40:, :] == 0)         # bottom rows see the lower half (+y up)
    assert np.all(A[:, :24] == 0)         # left columns see the lower x half
    zero = tf.copy()
    zero[:, 3] = 0
    assert np.all(oracle.render(vol, zero, cam, 64, 64) == 0)


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_render_skip_equals_full_march(seed):
    dims = [(64, 64, 64), (37, 50, 29), (45, 33, 52), (64, 40, 24)][seed]
    B = [8, 8, 16, 8][seed]
    vol = synth.blobs_u8(dims, seed=40 + seed, n_blobs=5)
    tf = synth.tf_random(seed, 256)
    mn, mx = oracle.brick_minmax(vol, B)
    flags = oracle.classify(mn, mx, vol.dtype, tf)
    assert 0 < flags.mean() < 1
    for ortho in (0, 1):
        if ortho:
            cam = synth.orthographic(dims, 48, 40, synth.view_direction(seed + 7))
        else:
            cam = synth.perspective(dims, 48, 40, synth.view_direction(seed + 7))
        full = oracle.render(vol, tf, cam, 48, 40)
        skip = oracle.render(vol, tf, cam, 48, 40, mode=1, flags=flags, B=B)
        assert full[..., 3].max() > 0.1
        assert np.array_equal(full, skip)


def test_render_pixel_list_matches_full_image():
    w = synth.c1_workload()
    img = oracle.render(w["vol"], w["tf"], w["cam"], w["W"], w["H"])
    pix = np.array([[0, 0], [127, 127], [64, 60], [3, 100]], np.int32)
    sub = oracle.render(w["vol"], w["tf"], w["cam"], w["W"], w["H"], pixels=pix)
    assert np.array_equal(sub, img[pix[:, 1], pix[:, 0]])


# ---------------------------------------------------------------------------
# k-d tree with the voxel-tight split cost (Sec. 3.2.2: one tight box per
# macro cell, unions of them for regions spanning several cells)
# ---------------------------------------------------------------------------

def _tight_union_volume(tb3, lo, hi):
    """half-voxel volume of the union of the boxes of bricks [lo, hi) (tb3:
    [z][y][x][6] boxes, empty = no visible cell), 0 without one"""
    sub = tb3[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]].reshape(-1, 6)
    sub = sub[(sub[:, 3] > sub[:, 0]) & (sub[:, 4] > sub[:, 1]) & (sub[:, 5] > sub[:, 2])]
    if len(sub) == 0:
        return 0
    ext = sub[:, 3:].max(0).astype(np.int64) - sub[:, :3].min(0).astype(np.int64)
    return int(np.prod(ext))


def check_kd_tight(t, flags, tboxes, B, dims, halting, max_leaf, bins=4):
    """Every rule of the build with the tight cost, recomputed by brute force
    over the boxes: regions and children stay brick-tight (prefix counts),
    every compared volume is the union volume in half-voxel units."""
    nb = oracle.brick_grid(dims, B)
    pc = PrefixCount(flags, nb)
    tb3 = np.asarray(tboxes, np.int64).reshape(nb[2], nb[1], nb[0], 6)
    m = len(t["axis"])
    if flags.sum() == 0:
        assert m == 0
        return
    assert m % 2 == 1
    vroot = _tight_union_volume(tb3, t["lo"][0], t["hi"][0])
    cover = np.zeros(nb[::-1], int)
    for i in range(m):
        lo, hi = [int(v) for v in t["lo"][i]], [int(v) for v in t["hi"][i]]
        V = _tight_union_volume(tb3, lo, hi)
        allowed = (10 * V > vroot) if halting == 0 else (V > 512 * 8)
        cands = []
        if allowed:
            for a in range(3):
                e = hi[a] - lo[a]
                if e < 2:
                    continue
                for p in sorted({lo[a] + (j * e) // bins for j in range(1, bins)} - {lo[a], hi[a]}):
                    l1, r0 = list(hi), list(lo)
                    l1[a], r0[a] = p, p
                    cands.append((_tight_union_volume(tb3, lo, l1) + _tight_union_volume(tb3, r0, hi), a, p))
        best = min(cands) if cands else None
        if t["axis"][i] < 0:
            assert best is None or best[0] >= V
            if best is not None and max_leaf > 0:
                assert V <= max_leaf ** 3 * 8
            cover[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] += 1
            continue
        a, p, c = int(t["axis"][i]), int(t["plane"][i]), int(t["first_child"][i])
        assert best is not None
        if best[0] < V:
            assert (a, p) == (best[1], best[2])
        else:
            assert max_leaf > 0 and V > max_leaf ** 3 * 8
            ext = [min(B * hi[q], dims[q]) - B * lo[q] if hi[q] - lo[q] >= 2 else -1 for q in range(3)]
            assert a == int(np.argmax(ext)) and p == lo[a] + (hi[a] - lo[a]) // 2
        for side, child in ((0, c), (1, c + 1)):
            rlo, rhi = list(lo), list(hi)
            if side == 0:
                rhi[a] = p
            else:
                rlo[a] = p
            tl, th = pc.tight(rlo, rhi)
            assert list(t["lo"][child]) == tl and list(t["hi"][child]) == th
    f3 = flags.reshape(nb[::-1]).astype(bool)
    assert np.all(cover <= 1) and np.all(cover[f3] == 1)


def test_kd_tight_cost_changes_the_plane():
    # four 8^3 bricks along x (32 x 8 x 8 voxels), bricks 0, 1 and 3 non-empty.
    # Brick cost: planes 1, 2, 3 cost 4, 3, 3 bricks against the root's 4 ->
    # split at 2 (tie with 3: smaller plane); the child [0, 2) would cost 2
    # bricks = its own volume -> leaf.  Voxel-tight boxes: brick 0 visible only
    # in x [0, 1), brick 1 only in x [15, 16), brick 3 everywhere (y, z full):
    # per unit of y-z area the root's union is [0, 32) = 32, plane 1 costs
    # 1 + (32 - 15) = 18, planes 2 and 3 cost 16 + 8 = 24 -> split at 1; the
    # right child [1, 4) (union [15, 32) = 17 > 512 / 64 = 8 voxels deep)
    # splits at 2 (1 + 8 = 9 < 17, tie with 3), and both its children
    # ([1, 2): 1, [3, 4): 8, not above 8) are leaves.
    flags = np.array([1, 1, 0, 1], np.uint8)
    tb = np.zeros((4, 6), np.int32)
    tb[0] = [0, 0, 0, 2, 16, 16]          # half-voxel units
    tb[1] = [30, 0, 0, 32, 16, 16]
    tb[3] = [48, 0, 0, 64, 16, 16]
    dims = (32, 8, 8)
    brick = oracle.kd(flags, 8, dims, 1, 0, 4)
    assert len(brick["axis"]) == 3 and brick["height"] == 2
    assert brick["axis"][0] == 0 and brick["plane"][0] == 2
    assert list(brick["lo"][1]) == [0, 0, 0] and list(brick["hi"][1]) == [2, 1, 1]
    assert list(brick["lo"][2]) == [3, 0, 0] and list(brick["hi"][2]) == [4, 1, 1]
    tight = oracle.kd(flags, 8, dims, 1, 0, 4, tight_boxes=tb)
    assert len(tight["axis"]) == 5 and tight["height"] == 3
    assert list(tight["axis"]) == [0, -1, 0, -1, -1]
    assert list(tight["plane"]) == [1, 0, 2, 0, 0]
    assert list(tight["first_child"]) == [1, -1, 3, -1, -1]
    assert [list(v) for v in tight["lo"]] == [[0, 0, 0], [0, 0, 0], [1, 0, 0], [1, 0, 0], [3, 0, 0]]
    assert [list(v) for v in tight["hi"]] == [[4, 1, 1], [1, 1, 1], [4, 1, 1], [2, 1, 1], [4, 1, 1]]
    check_kd_tight(tight, flags, tb, 8, dims, 1, 0)


def test_kd_tight_cost_without_visible_cells_is_one_leaf():
    # flagged bricks whose cells are all invisible: every tight volume is 0,
    # so nothing splits (0 is not below 0) and the root is the only node
    flags = np.ones(8, np.uint8)
    tb = np.zeros((8, 6), np.int32)
    for halting in (0, 1):
        t = oracle.kd(flags, 8, (16, 16, 16), halting, 0, 4, tight_boxes=tb)
        assert len(t["axis"]) == 1 and t["axis"][0] == -1


def test_kd_tight_cost_full_boxes_equal_brick_cost():
    # when every flagged brick's tight box is the whole brick, the unions are
    # the brick-tight boxes and every volume is 8x the brick cost's: the trees
    # are identical
    vol = synth.blobs_u8((48, 40, 56), seed=41, n_blobs=5)
    mn, mx = oracle.brick_minmax(vol, 8)
    flags = oracle.classify(mn, mx, vol.dtype, synth.tf_ramp(256, start=0.3))
    nb = oracle.brick_grid((48, 40, 56), 8)
    tb = np.zeros((flags.size, 6), np.int32)
    for b in np.flatnonzero(flags):
        x, y, z = b % nb[0], (b // nb[0]) % nb[1], b // (nb[0] * nb[1])
        lo = np.array([x, y, z]) * 8
        hi = np.minimum(lo + 8, [48, 40, 56])
        tb[b] = np.concatenate([2 * lo, 2 * hi])
    for halting, mls in ((0, 0), (1, 0), (1, 16)):
        a = oracle.kd(flags, 8, (48, 40, 56), halting, mls)
        b = oracle.kd(flags, 8, (48, 40, 56), halting, mls, tight_boxes=tb)
        for k in ("lo", "hi", "axis", "plane", "first_child"):
            assert np.array_equal(a[k], b[k]), (halting, mls, k)


@pytest.mark.parametrize("bins", [2, 4, 8])
@pytest.mark.parametrize("halting,max_leaf", [(0, 0), (1, 0), (1, 16)])
@pytest.mark.parametrize("seed,dims,B", [(0, (48, 40, 56), 8), (1, (37, 29, 33), 4), (2, (64, 48, 40), 16)])
def test_kd_tight_cost_rules(seed, dims, B, halting, max_leaf, bins):
    vol = synth.blobs_u8(dims, seed=60 + seed, n_blobs=6)
    tf = synth.tf_random(70 + seed, 256)
    mn, mx = oracle.brick_minmax(vol, B)
    flags = oracle.classify(mn, mx, vol.dtype, tf)
    tb = oracle.tight_boxes(vol, B, tf, flags)
    t = oracle.kd(flags, B, dims, halting, max_leaf, bins, tight_boxes=tb)
    check_kd_tight(t, flags, tb, B, dims, halting, max_leaf, bins)
