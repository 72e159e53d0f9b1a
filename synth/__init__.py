"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module only *generates inputs*: volumes, transfer functions and camera
bases.  It holds none of the method's arithmetic (no classification, no
hierarchy, no marching), so both the device library and the CPU oracle can be
fed from it without sharing any of the computation under test.

Arrays are numpy, volumes are indexed [z][y][x] (x fastest in memory),
transfer functions are (N, 4) float32 RGBA, cameras are dicts with the FP32
basis the C ABI takes: ``ortho``, ``eye``, ``dir00``, ``du``, ``dv``.

The paper's data sets (Sec. 4.2) are not available here; these generators
stand in for them with the same size and occupancy regime: sparse blobs,
thresholded fractal noise, thin tubes.
"""
from __future__ import annotations

import math

import numpy as np


# --------------------------------------------------------------------------
# volumes
# --------------------------------------------------------------------------

def blobs_u8(dims_xyz=(64, 64, 64), n_blobs=6, seed=1, sigma=(4.0, 8.0), cut=60,
             centre_range=(0.2, 0.8)):
    """Sum of Gaussian blobs at voxel centres, scaled to u8, values below
    ``cut`` zeroed (about 10 % non-zero voxels at 64^3 with the defaults)."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = dims_xyz
    dims = np.array([nx, ny, nz], np.float64)
    centres = rng.uniform(centre_range[0], centre_range[1], size=(n_blobs, 3)) * dims
    sig = rng.uniform(sigma[0], sigma[1], size=n_blobs)
    x = np.arange(nx) + 0.5
    y = np.arange(ny) + 0.5
    z = np.arange(nz) + 0.5
    acc = np.zeros((nz, ny, nx), np.float64)
    for c, s in zip(centres, sig):
        gx = np.exp(-((x - c[0]) ** 2) / (2 * s * s))
        gy = np.exp(-((y - c[1]) ** 2) / (2 * s * s))
        gz = np.exp(-((z - c[2]) ** 2) / (2 * s * s))
        acc += gz[:, None, None] * gy[None, :, None] * gx[None, None, :]
    v = np.minimum(255.0, np.floor(255.0 * acc + 0.5))
    v[v < cut] = 0
    return v.astype(np.uint8)


def _interp_axis(lat, axis, n, spacing):
    """Smoothstep-weighted linear interpolation of a lattice along one axis,
    evaluated at voxel centres (i + 0.5) / spacing."""
    u = (np.arange(n) + 0.5) / spacing
    i = np.floor(u).astype(np.int64)
    f = u - i
    w = f * f * (3.0 - 2.0 * f)
    a = np.take(lat, i, axis=axis)
    b = np.take(lat, i + 1, axis=axis)
    shape = [1, 1, 1]
    shape[axis] = n
    w = w.reshape(shape)
    return a * (1.0 - w) + b * w


def fractal_noise(dims_xyz=(512, 512, 512), seed=2, spacings=(64, 32, 16, 8, 4),
                  keep_fraction=0.05):
    """Fractal value noise (octaves at the given lattice spacings, amplitude
    halved per octave, smoothstep-weighted trilinear), normalised to [0,1],
    then thresholded at its (1-keep_fraction) quantile tau:
    v = 0 where f < tau, else (f - tau) / (max - tau).  Returns float32."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = dims_xyz
    acc = np.zeros((nz, ny, nx), np.float64)
    amp = 1.0
    for sp in spacings:
        L = [int(math.ceil(n / sp)) + 2 for n in (nx, ny, nz)]
        lat = rng.uniform(0.0, 1.0, size=(L[2], L[1], L[0]))
        t = _interp_axis(lat, 2, nx, sp)
        t = _interp_axis(t, 1, ny, sp)
        t = _interp_axis(t, 0, nz, sp)
        acc += amp * t
        del t
        amp *= 0.5
    lo, hi = acc.min(), acc.max()
    acc -= lo
    acc /= (hi - lo)
    flat = acc.reshape(-1)
    k = int(round((1.0 - keep_fraction) * (flat.size - 1)))
    tau = np.partition(flat, k)[k]
    top = flat.max()
    out = np.where(acc < tau, 0.0, (acc - tau) / (top - tau))
    return out.astype(np.float32)


def tubes(dims_xyz=(128, 128, 128), n_tubes=24, seed=3, radius=(2.0, 6.0), n_ctrl=6,
          samples_per_segment=32, dtype=np.float32):
    """Thin tubes along random Catmull-Rom curves (vessel-like), value 1 at
    the axis falling linearly to 0 at the radius.  float32 unless dtype says
    otherwise (u16 is scaled to 65535)."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = dims_xyz
    dims = np.array([nx, ny, nz], np.float64)
    vol = np.zeros((nz, ny, nx), np.float32)
    for _ in range(n_tubes):
        ctrl = rng.uniform(0.1, 0.9, size=(n_ctrl, 3)) * dims
        r = rng.uniform(radius[0], radius[1])
        pts = []
        for j in range(1, n_ctrl - 2):
            p0, p1, p2, p3 = ctrl[j - 1], ctrl[j], ctrl[j + 1], ctrl[j + 2]
            for t in np.linspace(0.0, 1.0, samples_per_segment, endpoint=False):
                t2, t3 = t * t, t * t * t
                pts.append(0.5 * ((2 * p1) + (-p0 + p2) * t + (2 * p0 - 5 * p1 + 4 * p2 - p3) * t2
                                  + (-p0 + 3 * p1 - 3 * p2 + p3) * t3))
        for p in pts:
            lo = np.maximum(np.floor(p - r - 1).astype(int), 0)
            hi = np.minimum(np.ceil(p + r + 1).astype(int), [nx, ny, nz])
            if np.any(hi <= lo):
                continue
            zz, yy, xx = np.meshgrid(np.arange(lo[2], hi[2]) + 0.5, np.arange(lo[1], hi[1]) + 0.5,
                                     np.arange(lo[0], hi[0]) + 0.5, indexing="ij")
            d = np.sqrt((xx - p[0]) ** 2 + (yy - p[1]) ** 2 + (zz - p[2]) ** 2)
            val = np.clip(1.0 - d / r, 0.0, 1.0).astype(np.float32)
            sl = vol[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]]
            np.maximum(sl, val, out=sl)
    if np.dtype(dtype) == np.uint16:
        return np.floor(vol.astype(np.float64) * 65535.0 + 0.5).astype(np.uint16)
    return vol.astype(dtype)


# --------------------------------------------------------------------------
# transfer functions
# --------------------------------------------------------------------------

def tf_ramp(N=256, start=0.3, peak=0.8):
    """Alpha 0 below ``start``, then a linear ramp to ``peak`` at 1; RGB ramps
    r = s, g = 1 - |2s - 1|, b = 1 - s (s = i / (N-1))."""
    s = np.arange(N, dtype=np.float64) / (N - 1)
    a = np.where(s < start, 0.0, peak * (s - start) / (1.0 - start))
    rgba = np.stack([s, 1.0 - np.abs(2.0 * s - 1.0), 1.0 - s, a], axis=1)
    return rgba.astype(np.float32)


def tf_random(seed, N=256, zero_below=(0.05, 0.5), min_gap=0.02):
    """A random piecewise-linear TF: 2-6 alpha control points in [a, 1] with
    alpha U[0,1], alpha forced to 0 on [0, a), a ~ U(zero_below); control
    points at least ``min_gap`` apart (bounds the TF slope); random PL RGB."""
    rng = np.random.default_rng(seed)
    a = rng.uniform(*zero_below)
    m = int(rng.integers(2, 7))
    while True:
        pos = np.sort(rng.uniform(a, 1.0, size=m))
        if np.all(np.diff(np.concatenate([[a], pos])) >= min_gap):
            break
    alpha = rng.uniform(0.0, 1.0, size=m)
    xs = np.concatenate([[a], pos])
    ys = np.concatenate([[0.0], alpha])
    s = np.arange(N, dtype=np.float64) / (N - 1)
    al = np.where(s < a, 0.0, np.interp(s, xs, ys))
    cpos = np.linspace(0.0, 1.0, 4)
    rgb = [np.interp(s, cpos, rng.uniform(0.0, 1.0, size=4)) for _ in range(3)]
    return np.stack(rgb + [al], axis=1).astype(np.float32)


# --------------------------------------------------------------------------
# cameras: the caller-side FP32 basis the ABI takes
# --------------------------------------------------------------------------

def _normalize(v):
    v = np.asarray(v, np.float64)
    return v / np.linalg.norm(v)


def _basis(forward, up=(0.0, 1.0, 0.0)):
    f = _normalize(forward)
    up = np.asarray(up, np.float64)
    if abs(np.dot(f, _normalize(up))) > 0.999:
        up = np.array([0.0, 0.0, 1.0])
    r = _normalize(np.cross(f, up))
    u = np.cross(r, f)
    return f, r, u


def _rot_y(v, deg):
    t = math.radians(deg)
    c, s = math.cos(t), math.sin(t)
    x, y, z = v
    return np.array([c * x + s * z, y, -s * x + c * z])


def view_direction(seed):
    """A seed-fixed unit direction from the volume centre towards the eye."""
    rng = np.random.default_rng(seed)
    v = rng.normal(size=3)
    return v / np.linalg.norm(v)


def perspective(dims_xyz, W, H, direction, fovy_deg=45.0, dist=1.6, orbit_deg=0.0):
    """Perspective camera at ``dist`` x (volume diagonal) from the centre
    along ``direction`` (rotated by ``orbit_deg`` about +y), looking at the
    centre, up = +y.  Pixel (x, y), y = 0 the top row, has the direction
    dir00 + (x+.5) du + (y+.5) dv."""
    dims = np.asarray(dims_xyz, np.float64)
    c = dims / 2.0
    diag = float(np.linalg.norm(dims))
    dirv = _rot_y(_normalize(direction), orbit_deg)
    eye = c + dist * diag * dirv
    f, r, u = _basis(c - eye)
    h = math.tan(math.radians(fovy_deg) / 2.0)
    w = h * W / H
    dir00 = f - w * r + h * u
    du = (2.0 * w / W) * r
    dv = -(2.0 * h / H) * u
    return dict(ortho=0, eye=eye.astype(np.float32), dir00=dir00.astype(np.float32),
                du=du.astype(np.float32), dv=dv.astype(np.float32))


def orthographic(dims_xyz, W, H, direction, dist=1.6, orbit_deg=0.0, zoom=1.0):
    """Orthographic camera looking at the centre from ``direction``; the view
    spans the volume diagonal / zoom vertically (the paper zooms so the volume
    fills the viewport).  Pixel (x, y) has origin eye + (x+.5) du + (y+.5) dv."""
    dims = np.asarray(dims_xyz, np.float64)
    c = dims / 2.0
    diag = float(np.linalg.norm(dims))
    dirv = _rot_y(_normalize(direction), orbit_deg)
    f, r, u = _basis(-dirv)
    hh = 0.5 * diag / zoom
    hw = hh * W / H
    eye = c - dist * diag * f - hw * r + hh * u
    du = (2.0 * hw / W) * r
    dv = -(2.0 * hh / H) * u
    return dict(ortho=1, eye=eye.astype(np.float32), dir00=f.astype(np.float32),
                du=du.astype(np.float32), dv=dv.astype(np.float32))


# --------------------------------------------------------------------------
# named workloads
# --------------------------------------------------------------------------

def c1_workload():
    """64^3 u8 blobs (~10 % non-zero), ramp TF, 8^3 bricks, 128x128
    perspective, step 0.5 voxel."""
    vol = blobs_u8((64, 64, 64), seed=1)
    return dict(vol=vol, tf=tf_ramp(256), brick=8, W=128, H=128, dt=0.5,
                cam=perspective((64, 64, 64), 128, 128, view_direction(1)))


def c2_camera(i, W=1920, H=1080, dims=(512, 512, 512)):
    """The camera of TF i in the 100-TF sequence: orbit 3.6 degrees per TF."""
    return perspective(dims, W, H, view_direction(2), orbit_deg=3.6 * i)


def c2_tfs(count=100, N=256):
    return [tf_random(1000 + i, N) for i in range(count)]


def menger_sponge(level=3, scale=3, value=200):
    """u8 Menger sponge of 3^level cells, each ``scale`` voxels wide: a solid
    cube with every cross-shaped tunnel removed at every level, so its empty
    space lies inside the volume (the paper's hard case for k-d builders)."""
    n = 3 ** level
    idx = np.arange(n)
    solid = np.ones((n, n, n), bool)
    for lv in range(level):
        d = (idx // (3 ** lv)) % 3 == 1
        cz, cy, cx = np.meshgrid(d, d, d, indexing="ij")
        holes = (cx & cy) | (cy & cz) | (cx & cz)
        solid &= ~holes
    vol = np.repeat(np.repeat(np.repeat(solid, scale, 0), scale, 1), scale, 2)
    return (vol * value).astype(np.uint8)


def _blob_volume_torch(dims, nb, density, rng, device, dtype="u8"):
    import torch
    nx, ny, nz = dims
    centres = rng.uniform(0.1, 0.9, size=(nb, 3)) * np.array(dims)
    sig = rng.uniform(0.04, 0.12, size=nb) * min(dims)
    x = torch.arange(nx, device=device, dtype=torch.float32) + 0.5
    y = torch.arange(ny, device=device, dtype=torch.float32) + 0.5
    z = torch.arange(nz, device=device, dtype=torch.float32) + 0.5
    acc = torch.zeros((nz, ny, nx), device=device, dtype=torch.float32)
    for c, s in zip(centres, sig):
        gx = torch.exp(-((x - float(c[0])) ** 2) / (2 * s * s))
        gy = torch.exp(-((y - float(c[1])) ** 2) / (2 * s * s))
        gz = torch.exp(-((z - float(c[2])) ** 2) / (2 * s * s))
        acc += gz[:, None, None] * gy[None, :, None] * gx[None, None, :]
    acc = acc / acc.max()
    flat = acc.reshape(-1)
    k = max(1, int(density * flat.numel()))
    # the k-th largest value, without sorting a billion voxels
    sample = flat[torch.randint(0, flat.numel(), (1 << 20,), device=device,
                                generator=torch.Generator(device=device).manual_seed(int(rng.integers(1 << 30))))]
    cut = torch.quantile(sample, 1.0 - density)
    if dtype == "f16":
        vol = torch.where(acc >= cut, acc, torch.zeros_like(acc)).to(torch.float16)
    else:
        vol = torch.where(acc >= cut, torch.clamp(acc * 255.0, 1.0, 255.0), torch.zeros_like(acc)).to(torch.uint8)
    del acc
    return vol.contiguous()


def tubes_torch(dims_xyz, fraction=0.02, seed=3, radius=(2.0, 6.0), n_ctrl=6, spacing=0.75, device="cuda",
                chunk=2048):
    """The tubes() recipe for large volumes, generated on `device` with torch:
    Catmull-Rom curves through random control points, value 1 on the axis
    falling linearly to 0 at the tube radius (max over overlapping tubes).
    Curve points are spaced at most `spacing` voxels apart so tubes stay
    continuous at any size; tubes are added until their estimated volume
    reaches `fraction` of the voxels.  Returns a float32 [nz, ny, nx] tensor."""
    import torch
    rng = np.random.default_rng(seed)
    nx, ny, nz = dims_xyz
    dims = np.array([nx, ny, nz], np.float64)
    target = fraction * float(nx) * ny * nz
    pts, rad = [], []
    filled = 0.0
    while filled < target:
        ctrl = rng.uniform(0.1, 0.9, size=(n_ctrl, 3)) * dims
        r = float(rng.uniform(radius[0], radius[1]))
        for j in range(1, n_ctrl - 2):
            p0, p1, p2, p3 = ctrl[j - 1], ctrl[j], ctrl[j + 1], ctrl[j + 2]
            fine = np.linspace(0.0, 1.0, 65)[:, None]
            def curve(t):
                t2, t3 = t * t, t * t * t
                return 0.5 * ((2 * p1) + (-p0 + p2) * t + (2 * p0 - 5 * p1 + 4 * p2 - p3) * t2
                              + (-p0 + 3 * p1 - 3 * p2 + p3) * t3)
            length = float(np.linalg.norm(np.diff(curve(fine), axis=0), axis=1).sum())
            n = max(2, int(np.ceil(length / spacing)))
            seg = curve(np.linspace(0.0, 1.0, n, endpoint=False)[:, None])
            pts.append(seg)
            rad.append(np.full(n, r))
            filled += np.pi * r * r * length           # non-zero voxels of the tube, overlaps ignored
    P = torch.from_numpy(np.concatenate(pts)).to(device=device, dtype=torch.float32)
    Rr = torch.from_numpy(np.concatenate(rad)).to(device=device, dtype=torch.float32)
    K = int(np.ceil(radius[1])) * 2 + 3
    off = torch.arange(K, device=device, dtype=torch.int64) - K // 2
    oz, oy, ox = torch.meshgrid(off, off, off, indexing="ij")
    offs = torch.stack([ox.reshape(-1), oy.reshape(-1), oz.reshape(-1)], 1)        # [K^3, 3] (x, y, z)
    vol = torch.zeros(nz * ny * nx, device=device, dtype=torch.float32)
    n_xyz = torch.tensor([nx, ny, nz], device=device, dtype=torch.int64)
    for i in range(0, P.shape[0], chunk):
        p = P[i:i + chunk]
        r = Rr[i:i + chunk]
        cell = torch.floor(p).to(torch.int64)[:, None, :] + offs[None]               # [c, K^3, 3]
        ok = ((cell >= 0) & (cell < n_xyz)).all(-1)
        d = torch.linalg.norm(cell.to(torch.float32) + 0.5 - p[:, None, :], dim=-1)
        val = torch.clamp(1.0 - d / r[:, None], 0.0, 1.0)
        ok &= val > 0
        idx = cell[..., 0] + nx * (cell[..., 1] + ny * cell[..., 2])
        vol.scatter_reduce_(0, idx[ok], val[ok], reduce="amax")
    return vol.view(nz, ny, nx)


def c3_workloads():
    """Large-volume precision cases: 1024^3 tubes (~2 % of voxels) stored as
    f32 and f16, and 2048^3 tubes stored as u16; 8^3 bricks."""
    return [dict(name="tubes1024", dims=(1024, 1024, 1024), fraction=0.02, seed=31, storage=("f32", "f16")),
            dict(name="tubes2048", dims=(2048, 2048, 2048), fraction=0.02, seed=32, storage=("u16",))]


def serving_volumes(count=16, seed=5, sizes=(128, 256, 512, 1024), device="cuda"):
    """Resident volumes for the serving workload: cubes of the given edge
    sizes, alternating u8 and f16 storage, blob sums at 1-20 % density."""
    rng = np.random.default_rng(seed)
    vols = []
    for i in range(count):
        n = int(sizes[i % len(sizes)])
        dt = "u8" if i % 2 == 0 else "f16"
        vol = _blob_volume_torch((n, n, n), int(rng.integers(3, 12)), float(rng.uniform(0.01, 0.2)), rng,
                                 device, dt)
        vols.append(dict(name=f"vol{i}", dims=(n, n, n), vol=vol, dtype=dt, tf=tf_random(seed * 1000 + i, 256)))
    return vols


def batch_workload(count=64, seed=4, image=(512, 512), device="cuda"):
    """Many uneven volumes, each with its own TF and camera: axis sizes drawn
    from {32, 64, 128, 256, 512} independently (anisotropic), u8 sums of
    Gaussian blobs with a cut chosen for 1-20 % non-empty voxels.  Volumes
    are generated on `device` with torch (separable Gaussians) from seeded
    parameters, so large batches build in seconds."""
    import torch
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        dims = tuple(int(v) for v in rng.choice([32, 64, 128, 256, 512], size=3))
        nb = int(rng.integers(3, 12))
        density = float(rng.uniform(0.01, 0.20))
        centres = rng.uniform(0.1, 0.9, size=(nb, 3)) * np.array(dims)
        sig = rng.uniform(0.04, 0.12, size=nb) * min(dims)
        nx, ny, nz = dims
        x = torch.arange(nx, device=device, dtype=torch.float32) + 0.5
        y = torch.arange(ny, device=device, dtype=torch.float32) + 0.5
        z = torch.arange(nz, device=device, dtype=torch.float32) + 0.5
        acc = torch.zeros((nz, ny, nx), device=device, dtype=torch.float32)
        for c, s in zip(centres, sig):
            gx = torch.exp(-((x - float(c[0])) ** 2) / (2 * s * s))
            gy = torch.exp(-((y - float(c[1])) ** 2) / (2 * s * s))
            gz = torch.exp(-((z - float(c[2])) ** 2) / (2 * s * s))
            acc += gz[:, None, None] * gy[None, :, None] * gx[None, None, :]
        acc = acc / acc.max()
        flat = acc.reshape(-1)
        k = max(1, int(density * flat.numel()))
        cut = torch.topk(flat, k).values[-1]
        vol = torch.where(acc >= cut, torch.clamp(acc * 255.0, 1.0, 255.0), torch.zeros_like(acc))
        vol = vol.to(torch.uint8).contiguous()
        tf = tf_random(seed * 1000 + i, 256)
        W, H = image
        cam = perspective(dims, W, H, view_direction(seed * 1000 + i))
        out.append(dict(dims=dims, vol=vol, tf=tf, cam=cam, W=W, H=H, density=density))
    return out
