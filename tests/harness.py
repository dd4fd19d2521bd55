"""Shared helpers of the parity tests: run the HIP path through the C ABI, run
the FP64 oracle on the same seeded inputs, build decision-margin masks and
compare.  Imports of torch and of the HIP binding are deferred so that CPU-only
tests can import this module."""
from __future__ import annotations

import numpy as np

from paper_2510_12174_amd import scenes

DELTA = 1e-5           # decision-margin threshold (relative)
IMG_TOL = 1e-4         # max-abs on every image channel
GRAD_REL = 1e-3        # |g - g_ref| <= 1e-3 |g_ref| + 1e-3 rms(g_ref)
PARAMS = ("mean", "quat", "log_scale", "opacity_logit", "mask_logit", "sh", "sem")
CHANNELS = dict(rgb=3, depth=1, kmap=1, normal=3, sem=None)


def say(*a):
    print(*a, flush=True)


# ------------------------------------------------------------------ workloads
def small_workload(kind, seed=0):
    """Reduced-size members of the workload families: same distributions, fewer
    Gaussians, smaller (ragged) images, so the oracle finishes in seconds."""
    if kind == "w1":
        return scenes.make_scene(1, r=seed)
    if kind == "w2s":
        cam = scenes.camera(200, 150, 187.5, 187.5, 100, 75,
                            np.array([[0.0, -1.0, 0.0], [0.0, 0.0, -1.0], [1.0, 0.0, 0.0]]), [0, 0, 2.5])
        return scenes.make_scene(2, r=seed, N=20000, views=[cam])
    if kind == "w2m":
        # the 640 x 480 view of workload 2 with 20,000 Gaussians: at 8 x 8 tiles
        # 4,800 tiles (13 bits, a two-pass tile sort)
        cam = scenes.camera(640, 480, 600, 600, 320, 240,
                            np.array([[0.0, -1.0, 0.0], [0.0, 0.0, -1.0], [1.0, 0.0, 0.0]]), [0, 0, 2.5])
        return scenes.make_scene(2, r=seed, N=20000, views=[cam])
    if kind == "w2c12":
        # 12 semantic channels: padded to 16 inside the kernels, so the padding
        # lanes of every channel block are exercised
        g, cams, o = small_workload("w2s", seed)
        g = dict(g)
        g["sem"] = np.ascontiguousarray(np.asarray(g["sem"]).reshape(g["N"], -1)[:, :12])
        g["C_o"] = 12
        return g, cams, o
    if kind == "w2c200":
        # 200 semantic channels (beyond one 128-channel forward pass and six
        # 32-channel backward passes): N(0, 1) logits from their own seed
        g, cams, o = small_workload("w2s", seed)
        g = dict(g)
        rng = np.random.Generator(np.random.PCG64(2200 + seed))
        g["sem"] = rng.standard_normal((g["N"], 200)).astype(np.float32)
        g["C_o"] = 200
        return g, cams, o
    if kind == "w3s":
        cam = scenes.camera(240, 136, 225, 225, 120, 68,
                            np.array([[0.0, -1.0, 0.0], [0.0, 0.0, -1.0], [1.0, 0.0, 0.0]]), [0, 0, 2.5])
        return scenes.make_scene(3, r=seed, N=30000, views=[cam])
    if kind == "w4s":
        g, cams, o = scenes.make_scene(4, r=seed, N=20000)
        small = []
        for v, (W, H) in enumerate([(96, 72), (120, 68), (130, 97)]):
            c = dict(cams[v])
            s = W / c["W"]
            c.update(W=W, H=H, fx=c["fx"] * s, fy=c["fy"] * s, cx=W / 2.0, cy=H / 2.0)
            small.append(c)
        return g, small, o
    if kind == "w5s":
        g, cams, o = scenes.make_scene(5, r=seed, N=30000)
        small = []
        for v in (0, 8):
            c = dict(cams[v])
            W, H = c["W"] // 10, c["H"] // 10
            s = W / c["W"]
            c.update(W=W, H=H, fx=c["fx"] * s, fy=c["fy"] * s, cx=W / 2.0, cy=H / 2.0)
            small.append(c)
        return g, small, o
    if kind == "wbig":
        # ten large Gaussians (sigma 25-50 px, centres up to 25 px outside the
        # view) with 128 channels: pixel offsets of up to ~180 px from the mean
        # inside one 8 x 8 block, through a first pass and a channel pass
        g, cams, o = scenes.tiny_scene(n=10, seed=11, W=160, H=120, C_o=128, sh_deg=1, f=120.0)
        rng = np.random.Generator(np.random.PCG64(4411 + seed))
        g = dict(g)
        mean = np.array(g["mean"], copy=True)
        mean[0] = rng.uniform(-2.2, 2.2, g["N"])
        mean[1] = rng.uniform(-1.7, 1.7, g["N"])
        g["mean"] = np.ascontiguousarray(mean, dtype=np.float32)
        g["log_scale"] = np.ascontiguousarray(np.asarray(g["log_scale"]) + 1.3, dtype=np.float32)
        return g, cams, o
    raise ValueError(kind)


# ------------------------------------------------------------------ GPU side
def stack_upstream(ups, C_o):
    import torch
    cat = lambda k: torch.from_numpy(np.concatenate([np.asarray(u[k], np.float32).reshape(-1) for u in ups])).cuda()
    return dict(rgb=cat("rgb"), depth=cat("depth"), kmap=cat("kmap"), normal=cat("normal"),
                sem=cat("sem") if C_o > 0 else None)


def unstack(out, cams, C_o):
    from paper_2510_12174_amd import unigs as U
    res = []
    views = {k: U.split_views(out[k], cams, c if c else C_o) for k, c in
             (("rgb", 3), ("depth", 1), ("kmap", 1), ("normal", 3), ("T_final", 1), ("n_contrib", 1))}
    if C_o > 0:
        views["sem"] = U.split_views(out["sem"], cams, C_o)
    for v, cam in enumerate(cams):
        d = {k: views[k][v].cpu().numpy() for k in views}
        for k in ("depth", "kmap", "T_final", "n_contrib"):
            d[k] = d[k].reshape(cam["H"], cam["W"])
        if C_o == 0:
            d["sem"] = np.zeros((0, cam["H"], cam["W"]), np.float32)
        res.append(d)
    return res


def gpu_run(g, cams, opts, ups=None, tile=(16, 16), batch=0, per_view=False, rast=None):
    """Forward (and backward when `ups` is given) through the C ABI.  Returns
    (per-view outputs, grads or None, rasterizer)."""
    import torch
    from paper_2510_12174_amd import unigs as U
    gd = U.to_device(g)
    C_o = int(g["C_o"])
    if rast is None:
        rast = U.Rasterizer(tile_w=tile[0], tile_h=tile[1], batch=batch, prune_Tk=float(opts.get("prune_Tk", 0.0)),
                            depth_mode=int(opts.get("depth_mode", 0)), sem_bf16x3=int(opts.get("sem_bf16x3", 0)))
    if not per_view:
        out = rast.forward(gd, cams)
        grads = None
        if ups is not None:
            grads = rast.backward(gd, out, stack_upstream(ups, C_o))
        torch.cuda.synchronize()
        outs = unstack(out, cams, C_o)
    else:
        outs, grads = [], (U.zeros_like_params(gd) if ups is not None else None)
        for v, cam in enumerate(cams):
            o = rast.forward(gd, [cam])
            if ups is not None:
                rast.backward(gd, o, stack_upstream([ups[v]], C_o), grads)
            torch.cuda.synchronize()
            outs += unstack(o, [cam], C_o)
    gr = None if grads is None else {k: grads[k].cpu().numpy().astype(np.float64) for k in PARAMS}
    return outs, gr, rast


# ------------------------------------------------------------------ oracle side
def oracle_forward(O, g, cams, opts):
    return O.forward_all(g, cams, opts)


def dilate_cross(mask, r):
    out = mask.copy()
    for s in range(1, r + 1):
        out[s:, :] |= mask[:-s, :]
        out[:-s, :] |= mask[s:, :]
        out[:, s:] |= mask[:, :-s]
        out[:, :-s] |= mask[:, s:]
    return out


def masks(O, g, cams, opts, outs, step2=2):
    """Per-view boolean masks of pixels to exclude: 'img' (forward decisions or a
    Gaussian with an ambiguous cull covers it), 'normal' (its own normal decisions
    or any stencil pixel excluded), 'grad' (img or the alpha clamp is marginal)."""
    res = []
    for cam, o in zip(cams, outs):
        bad = o["margin"] < DELTA
        P = O.project(g, cam, opts)
        amb = np.nonzero(P["ambiguous"] & (P["depth"] > 0))[0]
        H, W = cam["H"], cam["W"]
        for i in amb:
            rx, ry = P["radius"][i] * 1.1 + 2
            mx, my = P["mean2d"][i]
            x0, x1 = int(max(0, np.floor(mx - rx))), int(min(W - 1, np.ceil(mx + rx)))
            y0, y1 = int(max(0, np.floor(my - ry))), int(min(H - 1, np.ceil(my + ry)))
            if x0 <= x1 and y0 <= y1:
                bad[y0:y1 + 1, x0:x1 + 1] = True
        nbad = dilate_cross(bad, step2) | (o["nmargin"] < DELTA)
        gbad = bad | (o["grad_margin"] < DELTA)
        res.append(dict(img=bad, normal=nbad, grad=gbad))
    return res


def gauss_exclusions(O, g, cams, opts):
    """Gaussians whose gradient is not comparable: an ambiguous cull/skip test or
    an SH colour within 1e-5 of its clamp in some view."""
    ex = np.zeros(int(g["N"]), bool)
    for cam in cams:
        P = O.project(g, cam, opts)
        ex |= P["ambiguous"].astype(bool)
        ex |= np.any(np.abs(P["rgb_raw"]) < DELTA, axis=1) & P["visible"].astype(bool)
    return ex


def masked_upstream(ups, ms):
    res = []
    for u, m in zip(ups, ms):
        d = {}
        for k in ("rgb", "depth", "kmap", "sem"):
            a = np.array(u[k], np.float32, copy=True)
            if a.ndim == 3:
                a[:, m["grad"]] = 0
            else:
                a[m["grad"]] = 0
            d[k] = a
        n = np.array(u["normal"], np.float32, copy=True)
        n[:, m["normal"] | m["grad"]] = 0
        d["normal"] = n
        res.append(d)
    return res


# ------------------------------------------------------------------ comparisons
def image_errors(gpu_outs, ora_outs, ms, normals=True):
    """Max-abs error per channel over pixels not excluded."""
    err = {}
    for go, oo, m in zip(gpu_outs, ora_outs, ms):
        ok = ~m["img"]
        for k in ("rgb", "depth", "kmap", "sem", "T_final"):
            a = np.asarray(go[k], np.float64)
            b = np.asarray(oo[k], np.float64)
            if a.size == 0:
                continue
            d = np.abs(a - b)
            d = d[:, ok] if d.ndim == 3 else d[ok]
            err[k] = max(err.get(k, 0.0), float(d.max()) if d.size else 0.0)
        if normals:
            okn = ~m["normal"]
            d = np.abs(np.asarray(go["normal"], np.float64) - oo["normal"])[:, okn]
            err["normal"] = max(err.get("normal", 0.0), float(d.max()) if d.size else 0.0)
    return err


def last_ids(rast, cams, tile, per_view_vals=None):
    """Id of the last contributor of every pixel from the GPU's n_contrib and its
    sorted tile lists (-1 where none)."""
    vals = rast.debug_buffer("vals").cpu().numpy().astype(np.int64)
    ranges = rast.debug_buffer("ranges").cpu().numpy().astype(np.int64)
    return vals, ranges


def gpu_last_id(n_contrib, vals, ranges, cam, tile_base, tile):
    H, W = cam["H"], cam["W"]
    tw, th = tile
    tx = (W + tw - 1) // tw
    v, u = np.mgrid[0:H, 0:W]
    t = tile_base + (v // th) * tx + (u // tw)
    n = np.asarray(n_contrib, np.int64).reshape(H, W)
    pos = ranges[t, 0] + n - 1
    out = np.where(n > 0, vals[np.clip(pos, 0, max(len(vals) - 1, 0))] if len(vals) else -1, -1)
    return out


def grad_errors(gpu, ora, exclude):
    """Per tensor: max over elements of |g - r| / (1e-3 |r| + 1e-3 rms(r)); a
    value <= 1 meets the tolerance."""
    res = {}
    for k in PARAMS:
        a = np.asarray(gpu[k], np.float64)
        b = np.asarray(ora[k], np.float64)
        if b.size == 0:
            continue
        keep = ~exclude
        if k == "sem":
            a, b = a[keep], b[keep]
        else:
            a, b = a[..., keep], b[..., keep]
        rms = float(np.sqrt(np.mean(b * b))) if b.size else 0.0
        tol = GRAD_REL * np.abs(b) + GRAD_REL * rms + 1e-30
        res[k] = float(np.max(np.abs(a - b) / tol)) if b.size else 0.0
    return res
