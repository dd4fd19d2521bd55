"""Seeded synthetic scenes, cameras and upstream gradients.

This module only draws random inputs and lays them out; it contains none of
the rasterizer's arithmetic, and both the HIP path and the FP64 oracle are fed
from it.  Every array is drawn with numpy's PCG64 generator in a fixed order
(means, log-scales, quaternions, opacity logits, SH, semantic logits, mask
logits, then cameras), in float64, and cast to float32, so that the two sides
see bit-identical inputs.

Layout (structure of arrays, float32, C-contiguous):
  mean          [3][N]        world position
  quat          [4][N]        (w, x, y, z), not normalised
  log_scale     [3][N]
  opacity_logit [N]
  mask_logit    [N]           gradient factor k = sigmoid(mask_logit)
  sh            [(deg+1)^2][3][N]
  sem           [N][C_o]      semantic logits

Workload families (Gaussian count, distribution, SH degree, channels, views):
  1  2,000 Gaussians uniform in [-1,1]^3, SH degree 0, 8 channels, one
     128x128 view at distance 3.
  2  100,000 Gaussians uniform in a 6x4x3 m box, SH degree 3, 32 channels,
     one 640x480 view from inside the box.
  3  500,000 Gaussians on 20 planar patches, SH degree 3, 64 channels, one
     1200x680 view.
  4  1,000,000 Gaussians on patches, SH 3, 32 channels, 16 views of mixed
     resolution.
  5  3,000,000 Gaussians on patches, SH 3, 128 channels, 8 views at
     1920x1080 plus 8 at 960x540, pruning skip enabled (T_k = 0.2).
"""
from __future__ import annotations

import numpy as np

BOX_LO = np.array([-3.0, -2.0, -1.5])
BOX_HI = np.array([3.0, 2.0, 1.5])

WORKLOADS = {
    1: dict(N=2000, dist="cube", log_scale=(-3.0, 0.5), sh_deg=0, C_o=8,
            views="single128", prune_Tk=0.0),
    2: dict(N=100_000, dist="box", log_scale=(-3.0, 0.5), sh_deg=3, C_o=32,
            views="single640", prune_Tk=0.0),
    3: dict(N=500_000, dist="patches", log_scale=(-4.0, 0.7), sh_deg=3, C_o=64,
            views="single1200", prune_Tk=0.0),
    4: dict(N=1_000_000, dist="patches", log_scale=(-4.0, 0.7), sh_deg=3, C_o=32,
            views="mixed16", prune_Tk=0.0),
    5: dict(N=3_000_000, dist="patches", log_scale=(-4.0, 0.7), sh_deg=3, C_o=128,
            views="hd16", prune_Tk=0.2),
}

WORKLOAD_NAMES = {
    1: "single-view 2k Gaussians, 128x128, SH0, 8 channels",
    2: "single-view 100k Gaussians, 640x480, SH3, 32 channels",
    3: "single-view 500k surface Gaussians, 1200x680, SH3, 64 channels",
    4: "batched 16 views (640x480/960x720/1200x680/1296x968), 1M surface Gaussians, SH3, 32 channels",
    5: "batched 16 views (8x1920x1080 + 8x960x540), 3M surface Gaussians, SH3, 128 channels, pruning skip",
}


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def camera(W, H, fx, fy, cx, cy, R, t, z_near=0.2):
    R = np.asarray(R, dtype=np.float64).reshape(3, 3)
    t = np.asarray(t, dtype=np.float64).reshape(3)
    return dict(W=int(W), H=int(H), fx=float(fx), fy=float(fy), cx=float(cx),
                cy=float(cy), R=R.astype(np.float32), t=t.astype(np.float32),
                z_near=float(z_near))


def look_at(centre, target, W, H, f, up=(0.0, 0.0, 1.0), z_near=0.2):
    """Pinhole camera at `centre` looking at `target`: rows of the world-to-camera
    rotation are x_c = z_c x up, y_c = z_c x x_c, z_c = forward."""
    centre = np.asarray(centre, np.float64)
    zc = np.asarray(target, np.float64) - centre
    zc /= np.linalg.norm(zc)
    xc = np.cross(zc, np.asarray(up, np.float64))
    xc /= np.linalg.norm(xc)
    yc = np.cross(zc, xc)
    R = np.stack([xc, yc, zc])
    t = -R @ centre
    return camera(W, H, f, f, W / 2.0, H / 2.0, R, t, z_near)


def _patches(rng, n_patches=20):
    lo, hi = BOX_LO + 0.5, BOX_HI - 0.5
    centres = lo + (hi - lo) * rng.random((n_patches, 3))
    normals = rng.standard_normal((n_patches, 3))
    normals /= np.linalg.norm(normals, axis=1, keepdims=True)
    helper = rng.standard_normal((n_patches, 3))
    e1 = helper - np.sum(helper * normals, axis=1, keepdims=True) * normals
    e1 /= np.linalg.norm(e1, axis=1, keepdims=True)
    e2 = np.cross(normals, e1)
    half = rng.uniform(0.25, 1.0, size=(n_patches, 2))
    return dict(centre=centres, normal=normals, e1=e1, e2=e2, half=half)


def _means(rng, dist, N):
    if dist == "cube":
        return rng.uniform(-1.0, 1.0, size=(N, 3)), None
    if dist == "box":
        return BOX_LO + (BOX_HI - BOX_LO) * rng.random((N, 3)), None
    if dist == "patches":
        P = _patches(rng)
        which = rng.integers(0, len(P["centre"]), size=N)
        a = rng.uniform(-1.0, 1.0, size=N) * P["half"][which, 0]
        b = rng.uniform(-1.0, 1.0, size=N) * P["half"][which, 1]
        off = rng.normal(0.0, 0.01, size=N)
        mu = (P["centre"][which] + a[:, None] * P["e1"][which]
              + b[:, None] * P["e2"][which] + off[:, None] * P["normal"][which])
        return mu, P
    raise ValueError(dist)


def _views(rng, kind, patches):
    if kind == "single128":
        return [camera(128, 128, 128, 128, 64, 64, np.eye(3), [0, 0, 3])]
    box_R = np.array([[0.0, -1.0, 0.0], [0.0, 0.0, -1.0], [1.0, 0.0, 0.0]])
    if kind == "single640":
        return [camera(640, 480, 600, 600, 320, 240, box_R, [0, 0, 2.5])]
    if kind == "single1200":
        return [camera(1200, 680, 1125, 1125, 600, 340, box_R, [0, 0, 2.5])]
    if kind in ("mixed16", "hd16"):
        if kind == "mixed16":
            res = [(640, 480), (960, 720), (1200, 680), (1296, 968)]
            sizes = [res[v % 4] for v in range(16)]
            focal = [0.9375 * w for (w, _) in sizes]
        else:
            sizes = [(1920, 1080)] * 8 + [(960, 540)] * 8
            focal = [1800.0] * 8 + [900.0] * 8
        lo = np.array([-2.4, -1.6, -1.2])
        hi = -lo
        cams = []
        for v in range(16):
            target = patches["centre"][v % len(patches["centre"])]
            while True:
                c = lo + (hi - lo) * rng.random(3)
                if np.linalg.norm(c - target) >= 0.5:
                    break
            W, H = sizes[v]
            cams.append(look_at(c, target, W, H, focal[v]))
        return cams
    raise ValueError(kind)


def make_scene(workload: int, r: int = 0, N: int | None = None, seed: int | None = None,
               views: list | None = None):
    """Scene for a workload family.  `N` overrides the Gaussian count (same
    distribution), `views` overrides the camera list.  Returns (gaussians, cameras,
    options) where gaussians is a dict of float32 SoA arrays."""
    spec = WORKLOADS[workload]
    seed = 1000 * workload + r if seed is None else seed
    rng = _rng(seed)
    n = spec["N"] if N is None else int(N)
    mu, patches = _means(rng, spec["dist"], n)
    ls = rng.normal(spec["log_scale"][0], spec["log_scale"][1], size=(n, 3))
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    op = rng.standard_normal(n)
    deg = spec["sh_deg"]
    nc = (deg + 1) ** 2
    if deg == 0:
        sh = rng.random((n, 1, 3))
    else:
        sh = rng.normal(0.0, 0.3, size=(n, nc, 3))
    sem = rng.standard_normal((n, spec["C_o"]))
    mask = rng.normal(2.0, 1.0, size=n)
    cams = _views(rng, spec["views"], patches) if views is None else views
    g = dict(
        N=n, sh_deg=deg, C_o=spec["C_o"],
        mean=np.ascontiguousarray(mu.T, dtype=np.float32),
        quat=np.ascontiguousarray(q.T, dtype=np.float32),
        log_scale=np.ascontiguousarray(ls.T, dtype=np.float32),
        opacity_logit=np.ascontiguousarray(op, dtype=np.float32),
        mask_logit=np.ascontiguousarray(mask, dtype=np.float32),
        sh=np.ascontiguousarray(np.transpose(sh, (1, 2, 0)), dtype=np.float32),
        sem=np.ascontiguousarray(sem, dtype=np.float32),
    )
    opts = dict(prune_Tk=spec["prune_Tk"])
    return g, cams, opts


def upstream(cams, C_o, seed, density=1.0, channels=("rgb", "depth", "kmap", "normal", "sem")):
    """Upstream gradients dL/d(output) ~ N(0,1) per output element, one dict per
    view, planar [C][H][W] float32.  With density < 1 only a seeded random subset
    of pixels carries non-zero weights (the same subset for every channel).
    Channels not listed are zero."""
    rng = _rng(seed + 500)
    out = []
    for cam in cams:
        H, W = cam["H"], cam["W"]
        d = {}
        sizes = dict(rgb=3, depth=1, kmap=1, normal=3, sem=C_o)
        for name in ("rgb", "depth", "kmap", "normal", "sem"):
            c = sizes[name]
            if name in channels:
                a = rng.standard_normal((c, H, W), dtype=np.float32)
            else:
                a = np.zeros((c, H, W), np.float32)
            d[name] = a
        if density < 1.0:
            keep = rng.random((H, W)) < density
            for name in d:
                d[name] *= keep[None]
        d["depth"] = d["depth"].reshape(H, W)
        d["kmap"] = d["kmap"].reshape(H, W)
        out.append(d)
    return out


def tiny_scene(n=3, seed=7, W=32, H=24, C_o=4, sh_deg=1, f=40.0):
    """Small handmade-scale scene (a few Gaussians in front of one camera)."""
    rng = _rng(seed)
    mu = np.stack([rng.uniform(-0.4, 0.4, n), rng.uniform(-0.3, 0.3, n),
                   rng.uniform(-0.3, 0.3, n)], axis=1)
    ls = rng.normal(-1.6, 0.3, size=(n, 3))
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    op = rng.normal(1.0, 1.0, n)
    nc = (sh_deg + 1) ** 2
    sh = rng.normal(0.0, 0.4, size=(n, nc, 3))
    sh[:, 0, :] += 1.0
    sem = rng.standard_normal((n, C_o))
    mask = rng.normal(2.0, 1.0, size=n)
    g = dict(
        N=n, sh_deg=sh_deg, C_o=C_o,
        mean=np.ascontiguousarray(mu.T, dtype=np.float32),
        quat=np.ascontiguousarray(q.T, dtype=np.float32),
        log_scale=np.ascontiguousarray(ls.T, dtype=np.float32),
        opacity_logit=np.ascontiguousarray(op, dtype=np.float32),
        mask_logit=np.ascontiguousarray(mask, dtype=np.float32),
        sh=np.ascontiguousarray(np.transpose(sh, (1, 2, 0)), dtype=np.float32),
        sem=np.ascontiguousarray(sem, dtype=np.float32),
    )
    cam = camera(W, H, f, f, W / 2.0, H / 2.0, np.eye(3), [0, 0, 2.5])
    return g, [cam], dict(prune_Tk=0.0)
