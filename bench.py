#!/usr/bin/env python3
"""Benchmark: forward+backward megapixels/s of the multimodal Gaussian
rasterizer (RGB, ray-ellipsoid depth, normals, semantics, gradient factor), the
batched form (all views in one captured HIP graph) against the per-view form
(sequential per-view calls), on one MI355X.

Prints ONE JSON line.  `value` is the batched form's whole-job throughput with
all inputs resident in HBM (workload 5 by default: 3M Gaussians, 128 channels,
16 views, 20.7 MP); `per_view` carries the per-view form; `step_ms` the
per-step distribution (median, p10, p90 of HIP-event times); `roofline`
reports the dominant kernel (timed live with HIP events on the launch stream)
against its roofline; `secondary` the 16-view 1M-Gaussian workload in FP32 and
with the opt-in split-bf16 semantic products; `cpu_baseline` is the FP64
oracle on a bounded sample of the same workload on the host cores, plus the
oracle's single-view workloads, and `parity` compares the timed outputs and a
sampled backward with the oracle's values on that sample.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload 5]
"""
from __future__ import annotations

import argparse
import ctypes as C
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "fwd+bwd megapixels/sec (all modalities), batched vs per-view, at oracle tolerance"
PEAK_FP32 = 157.3e12   # MI355X FP32 vector (and FP32 matrix), FLOP/s
PEAK_HBM = 8.0e12      # MI355X HBM3E, B/s
STAGES = ["project", "bin_sort", "render_fwd", "normal_fwd", "normal_bwd", "render_bwd", "project_bwd"]
RENDER_SOURCES = "render_f32.hip,render_common.h"
KERNEL_SOURCE = {"project": "project.hip", "bin_sort": "binsort.hip", "render_fwd": RENDER_SOURCES,
                 "normal_fwd": "normal.hip", "normal_bwd": "normal.hip", "render_bwd": RENDER_SOURCES,
                 "project_bwd": "project.hip"}
IMG_TOL, GRAD_REL, DELTA = 1e-4, 1e-3, 1e-5


def log(*a):
    print(*a, file=sys.stderr, flush=True)


class HipEvents:
    """Raw hipEvent_t handles (recorded by the library on its launch stream)."""

    def __init__(self):
        self.L = C.CDLL("libamdhip64.so")
        self.L.hipEventElapsedTime.argtypes = [C.POINTER(C.c_float), C.c_void_p, C.c_void_p]
        self.L.hipEventSynchronize.argtypes = [C.c_void_p]
        self.L.hipEventDestroy.argtypes = [C.c_void_p]

    def create(self):
        e = C.c_void_p()
        assert self.L.hipEventCreate(C.byref(e)) == 0
        return e

    def sync(self, e):
        assert self.L.hipEventSynchronize(e) == 0

    def ms(self, a, b):
        t = C.c_float()
        assert self.L.hipEventElapsedTime(C.byref(t), a, b) == 0
        return float(t.value)


def pct(xs, q):
    return float(np.percentile(np.asarray(xs, np.float64), q))


def algorithmic(N, V_rec, P, Px, C_o, sh_deg, F_eval, F_contrib):
    """Compulsory HBM bytes of one fwd+bwd step and per-kernel FLOPs."""
    S_h = 3 * (sh_deg + 1) ** 2
    Bp = 4 * N * (11 + S_h + C_o + 1)
    b = (3 * Bp + 64 * V_rec * 2 + 64 * V_rec * 2 + 44 * P + Px * (4 * (8 + C_o) + 8) + Px * 4 * (8 + C_o)
         + Px * 24)
    f_fwd = 12 * F_eval + F_contrib * (2 * (C_o + 5) + 24)
    f_bwd = 12 * F_eval + F_contrib * (4 * (C_o + 5) + 80)
    return b, f_fwd, f_bwd


def measured_copy_bandwidth(torch, nbytes=1 << 30, reps=10):
    """Device-to-device copy rate (bytes read + written per second, median of
    `reps` copies of `nbytes`): the attainable-bandwidth reference beside the
    8 TB/s specification."""
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1) * 1e-3)
    del a, b
    torch.cuda.empty_cache()
    return 2 * nbytes / float(np.median(ts))


def binsort_bytes(R, P, tiles):
    """Algorithmic HBM bytes of the binning and sorting stage: the stable depth
    sort of the R visible records (4 passes of 8 bits: a 4-byte key read for
    the histogram, key and index read and written by the scatter), the two
    binning walks over the sorted records (index, rectangle and the 32 bytes of
    the culling record read; counts written, then the P (tile, index) pairs),
    the stable tile sort of the pairs (as many passes as 9-bit digits cover the
    tile ids: histogram read, pair read and written) and the per-tile ranges."""
    dp = 4
    tp = -(-max(tiles - 1, 0).bit_length() // 9)
    return (R * dp * (4 + 16) + 2 * R * (4 + 8 + 32) + R * 8 + P * 8 + tp * P * (4 + 16) + P * 4 + tiles * 8), tp


def source_sha(name):
    h = hashlib.sha256()
    for f in KERNEL_SOURCE[name].split(","):
        h.update(open(os.path.join(ROOT, "paper_2510_12174_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def profile_entry(fname, name, workload):
    """Entry of a committed counter summary taken on the current kernel source
    (None otherwise)."""
    p = os.path.join(ROOT, "profiles", fname)
    if not os.path.exists(p):
        return None
    d = json.load(open(p)).get(f"{name}@w{workload}")
    if not d or d.get("source_sha") != source_sha(name):
        return None
    return d


def stage_launches(stage, C_o, bf16):
    """Kernel launches that make up one compositing stage: the FP32 matrix-core
    kernels take the semantic channels in passes (forward: up to 64 per pass,
    backward: 32 when there are at most 32, else 64), the first pass also doing
    the colour, depth and alpha work."""
    if stage not in ("render_fwd", "render_bwd") or C_o <= 8 or (bf16 and C_o <= 32):
        return 1
    per = 64 if stage == "render_fwd" else (32 if C_o <= 32 else 64)
    return -(-C_o // per)


def tile_balance(clk):
    """Load balance of one compositing launch from its per-tile workgroup start
    and end times (100 MHz ticks): the launch span, the tail after the last
    tile started (the time the hardware dispatch can no longer fill the
    machine), and the tile-duration distribution."""
    st, en = clk[:, 0].astype(np.int64), clk[:, 1].astype(np.int64)
    span = float(en.max() - st.min())
    tail = float(en.max() - st.max())
    dur = (en - st).astype(np.float64)
    return dict(tiles=int(clk.shape[0]), span_ms=round(span / 1e5, 3), tail_ms=round(tail / 1e5, 3),
                tail_frac=round(tail / span, 4) if span > 0 else None,
                tile_ms=dict(median=round(pct(dur, 50) / 1e5, 4), p99=round(pct(dur, 99) / 1e5, 4),
                             max=round(float(dur.max()) / 1e5, 4)))


def device_upstream(torch, Px, C_o, seed):
    """Upstream gradients N(0, 1) per output element, drawn on the device."""
    gen = torch.Generator(device="cuda").manual_seed(seed)
    f = lambda n: torch.randn(n, device="cuda", generator=gen)
    return dict(rgb=f(3 * Px), depth=f(Px), kmap=f(Px), normal=f(3 * Px), sem=f(C_o * Px) if C_o else None)


def time_replays(torch, rast, steps, warmup):
    """Warm-up replays, then `steps` timed replays bracketed by device
    synchronisation: returns (wall ms per step, per-step HIP-event ms list)."""
    for _ in range(warmup):
        rast.replay()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for a, b in evs:
        a.record()
        rast.replay()
        b.record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps * 1e3
    return wall, [a.elapsed_time(b) for a, b in evs]


def per_view_rate(torch, U, g, cams, out, up, grads, opts, tune, C_o, steps, warmup, bf16):
    """V sequential project -> bin_sort (pair count read back) -> render_fwd ->
    render_bwd calls per step; returns ms per step."""
    pr = U.Rasterizer(prune_Tk=float(opts["prune_Tk"]), tile_w=tune.tile_w, tile_h=tune.tile_h, batch=tune.batch,
                      sem_bf16x3=int(bf16))
    off = U.pixel_offsets(cams)
    views = []
    for v, cam in enumerate(cams):
        a, b = off[v], off[v + 1]
        sl = lambda t, c: None if t is None else t[c * a:c * b]
        views.append(([cam], {k: sl(out[k], c) for k, c in (("rgb", 3), ("depth", 1), ("kmap", 1), ("normal", 3),
                                                            ("sem", C_o), ("T_final", 1), ("n_contrib", 1))},
                      {k: sl(up[k], c) for k, c in (("rgb", 3), ("depth", 1), ("kmap", 1), ("normal", 3),
                                                    ("sem", C_o))}))

    def step():
        for t in grads.values():
            t.zero_()
        for cv, ov, uv in views:
            pr.forward(g, cv, ov)
            pr.backward(g, ov, uv, grads)

    for _ in range(max(1, warmup)):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps * 1e3


def secondary_workload(torch, U, scenes, wl, steps, warmup):
    """The 16-view 1M-Gaussian workload: batched and per-view in FP32, and the
    batched step with the split-bf16 semantic products (dtype bf16x3)."""
    g_np, cams, opts = scenes.make_scene(wl)
    C_o = int(g_np["C_o"])
    Px = sum(c["W"] * c["H"] for c in cams)
    g = U.to_device(g_np)
    del g_np
    up = device_upstream(torch, Px, C_o, 1000 * wl)
    out = U.alloc_outputs(cams, C_o)
    grads = U.zeros_like_params(g)
    res = dict(workload=scenes.WORKLOAD_NAMES[wl], megapixels=round(Px / 1e6, 3))
    for name, bf16 in (("f32", False), ("bf16x3", True)):
        rast = U.Rasterizer(prune_Tk=float(opts["prune_Tk"]), sem_bf16x3=int(bf16))
        tuned = rast.autotune(g, cams, out, up, grads, cache=False)
        rast.capture_step(g, cams, out, up, grads)
        wall, ev = time_replays(torch, rast, steps, warmup)
        d = dict(dtype=name, value=round(Px / wall / 1e3, 2), unit="MP/s", ms_per_step=round(wall, 3),
                 step_ms=dict(median=round(pct(ev, 50), 3), p10=round(pct(ev, 10), 3), p90=round(pct(ev, 90), 3)),
                 tile=f"{tuned['tile_w']}x{tuned['tile_h']}", batch=int(tuned["batch"]))
        if not bf16:
            t_pv = per_view_rate(torch, U, g, cams, out, up, grads, opts, rast.opts, C_o, steps, warmup, False)
            d["per_view"] = dict(value=round(Px / t_pv / 1e3, 2), unit="MP/s", ms_per_step=round(t_pv, 3))
        res[name] = d
        del rast
    return res


# ------------------------------------------------------------------ CPU leg
def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.lower().startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _band(H, rows):
    pm = np.zeros(H, bool)
    r0 = max(0, H // 2 - rows // 2)
    pm[r0:r0 + rows] = True
    return pm


def cpu_baseline(torch, U, g_np, cams, opts, rast, out, budget_s=15.0):
    """FP64 oracle (forward + normals + backward) timed on a bounded sample of
    the workload (a band of central rows of the first view, sized from a short
    calibration run to about budget_s seconds), the oracle's single-view
    workloads (1 and 2 whole, 3 on a row band; medians of 3; workload 1 also at
    one thread), and the parity of the timed step's outputs with the oracle on
    the sample: images (rgb, depth, K, semantics), normals on the GPU's own
    depth, and the gradients of a backward whose upstream is confined to the
    sample (normal upstream zero; normals are compared stage-wise)."""
    from oracle import oracle as O
    from paper_2510_12174_amd import scenes
    S = O._Scene(g_np)
    C_o = int(g_np["C_o"])
    cam = cams[0]
    H, W = cam["H"], cam["W"]

    def run(rows, normal_up=True):
        band = _band(H, rows)
        pm = np.zeros((H, W), np.uint8)
        pm[band] = 1
        up = scenes.upstream([cam], C_o, seed=4242)[0]
        up = {k: (np.where(pm[None] > 0, u, 0) if u.ndim == 3 else np.where(pm > 0, u, 0)).astype(np.float32)
              for k, u in up.items()}
        if not normal_up:
            up["normal"][:] = 0
        t = time.perf_counter()
        o = O.render(S, cam, opts, path=1, pixmask=pm)
        O.normals(o["depth"], cam, opts, pixmask=pm)
        gr, _ = O.backward(S, cam, up, o["depth"], opts, path=1, pixmask=pm)
        return time.perf_counter() - t, int(pm.sum()), pm, o, up, gr

    t1, p1 = run(4)[:2]
    t2, p2 = run(24)[:2]
    per_px = max((t2 - t1) / max(p2 - p1, 1), 1e-9)
    fixed = max(t1 - p1 * per_px, 0.0)
    rows = int(min(H, max(8, (budget_s - fixed) / (per_px * W))))
    # the timed sample: its upstream excludes the normal branch, so that the
    # same band's gradients are comparable with a GPU backward (see parity)
    t, px, pm, o, up_np, gr_ref = run(rows, normal_up=False)
    res = dict(value=round(px / t / 1e6, 5), unit="MP/s", cores=O.max_threads(), kind="oracle",
               cpu_model=_cpu_model(), nproc=os.cpu_count(),
               sample=f"view 0 ({W}x{H}) {rows} central rows = {px} pixels, fwd+normals+bwd, {t:.1f} s")

    # single-view workloads of the oracle
    cfg = {}
    for wl, band_rows in ((1, None), (2, None), (3, 96)):
        g1, c1, o1 = scenes.make_scene(wl)
        S1 = O._Scene(g1)
        cm = c1[0]
        pm1 = None
        if band_rows:
            pm1 = np.zeros((cm["H"], cm["W"]), np.uint8)
            pm1[_band(cm["H"], band_rows)] = 1
        u1 = scenes.upstream([cm], int(g1["C_o"]), seed=1000 * wl)[0]

        def once():
            tt = time.perf_counter()
            oo = O.render(S1, cm, o1, path=1, pixmask=pm1)
            O.normals(oo["depth"], cm, o1, pixmask=pm1)
            O.backward(S1, cm, u1, oo["depth"], o1, path=1, pixmask=pm1)
            return time.perf_counter() - tt

        ts = [once() for _ in range(3)]
        npx = int(pm1.sum()) if pm1 is not None else cm["W"] * cm["H"]
        cfg[f"workload{wl}"] = dict(mp_per_s=round(npx / float(np.median(ts)) / 1e6, 4),
                                    median_s=round(float(np.median(ts)), 3), pixels=npx,
                                    sample="whole view" if pm1 is None else f"{band_rows} central rows")
        if wl == 1:
            O.set_threads(1)
            ts1 = [once() for _ in range(3)]
            O.set_threads(res["cores"])
            cfg["workload1_one_thread"] = dict(mp_per_s=round(npx / float(np.median(ts1)) / 1e6, 4),
                                               median_s=round(float(np.median(ts1)), 3))
    res["single_view_workloads"] = cfg

    # parity of the timed step on the sample
    parity = dict(pixels=px, tol=dict(image=IMG_TOL, grad_rel=GRAD_REL))
    ok_px = (o["margin"] >= DELTA) & (pm > 0)
    P = O.project(S, cam, opts)
    amb = P["ambiguous"].astype(bool)
    for i in np.nonzero(amb & (P["depth"] > 0))[0]:
        rx, ry = P["radius"][i] * 1.1 + 2
        mx, my = P["mean2d"][i]
        ok_px[max(0, int(my - ry)):max(0, int(my + ry) + 1), max(0, int(mx - rx)):max(0, int(mx + rx) + 1)] = False
    Pv = W * H
    gd = out["depth"][:Pv].cpu().numpy().reshape(H, W)
    maps = dict(rgb=(out["rgb"][:3 * Pv].cpu().numpy().reshape(3, H, W), o["rgb"]),
                depth=(gd, o["depth"]), kmap=(out["kmap"][:Pv].cpu().numpy().reshape(H, W), o["kmap"]))
    if C_o:
        maps["sem"] = (out["sem"][:C_o * Pv].cpu().numpy().reshape(C_o, H, W), o["sem"])
    img = {}
    for k, (a, b) in maps.items():
        d = np.abs(np.asarray(a, np.float64) - b)
        d = d[:, ok_px] if d.ndim == 3 else d[ok_px]
        img[k] = float(d.max()) if d.size else 0.0
    parity["image_max_abs"] = img
    parity["masked_pixels"] = int(((pm > 0) & ~ok_px).sum())
    nrm = O.normals(gd, cam, opts, pixmask=pm)
    okn = (nrm["margin"] >= DELTA) & (pm > 0)
    gn = out["normal"][:3 * Pv].cpu().numpy().reshape(3, H, W)
    parity["normal_stage_max_abs"] = float(np.abs(gn - nrm["normal"])[:, okn].max()) if okn.any() else 0.0
    # gradients: a GPU backward with the sample's upstream (zero on masked pixels)
    gmask = ok_px & (o["grad_margin"] >= DELTA)
    Px = out["depth"].numel()
    upd = dict(rgb=torch.zeros(3 * Px, device="cuda"), depth=torch.zeros(Px, device="cuda"),
               kmap=torch.zeros(Px, device="cuda"), normal=torch.zeros(3 * Px, device="cuda"),
               sem=torch.zeros(C_o * Px, device="cuda") if C_o else None)
    upm = {}
    for k, c in (("rgb", 3), ("depth", 1), ("kmap", 1), ("sem", C_o)):
        if c == 0:
            continue
        a = np.ascontiguousarray(np.asarray(up_np[k], np.float32).reshape(c, H, W) * gmask[None])
        upm[k] = a
        upd[k][:c * Pv] = torch.from_numpy(a.reshape(-1)).cuda()
    ref_up = dict(rgb=upm["rgb"], depth=upm["depth"][0], kmap=upm["kmap"][0], normal=np.zeros((3, H, W), np.float32),
                  sem=upm.get("sem", np.zeros((0, H, W), np.float32)))
    gd_t = U.to_device(g_np)
    o2 = rast.forward(gd_t, cams)
    grads = rast.backward(gd_t, o2, upd)
    torch.cuda.synchronize()
    ref, _ = O.backward(S, cam, ref_up, o["depth"], opts, path=1, pixmask=pm)
    ex = amb | (np.any(np.abs(P["rgb_raw"]) < DELTA, axis=1) & P["visible"].astype(bool))
    gerr = {}
    for k in ("mean", "quat", "log_scale", "opacity_logit", "mask_logit", "sh", "sem"):
        a = grads[k].cpu().numpy().astype(np.float64)
        b = np.asarray(ref[k], np.float64)
        if b.size == 0:
            continue
        keep = ~ex
        a, b = (a[keep], b[keep]) if k == "sem" else (a[..., keep], b[..., keep])
        rms = float(np.sqrt(np.mean(b * b))) if b.size else 0.0
        tol = GRAD_REL * np.abs(b) + GRAD_REL * rms + 1e-30
        gerr[k] = round(float(np.max(np.abs(a - b) / tol)), 4)
    parity["grad_err_over_tol"] = gerr
    parity["ok"] = bool(all(v <= IMG_TOL for v in img.values()) and parity["normal_stage_max_abs"] <= IMG_TOL
                        and all(v <= 1.0 for v in gerr.values()))
    del gr_ref, gd_t, o2, grads
    return res, parity


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", type=int, default=5)
    ap.add_argument("--secondary", type=int, default=4, help="second workload reported (0: none)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-per-view", action="store_true")
    ap.add_argument("--no-forward-only", action="store_true")
    ap.add_argument("--no-prune", action="store_true")
    ap.add_argument("--no-loss", action="store_true")
    ap.add_argument("--no-depth-modes", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--tile", default=None, help="force a tile shape, e.g. 16x16")
    ap.add_argument("--batch", type=int, default=0, help="force the LDS batch (with --tile)")
    ap.add_argument("--sem-bf16x3", action="store_true",
                    help="9..32 channels: split-bf16 semantic products (reported as dtype bf16x3)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one plain 1 GiB device copy first (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the rasterizer's multi-GPU form (views sharded "
              "across GPUs with one gradient all-reduce) is not implemented.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2510_12174_amd import scenes
    from paper_2510_12174_amd import unigs as U

    if not os.path.exists(U.LIB):
        raise SystemExit("libunigs.so is not built: run python __graft_entry__.py")
    wl = args.workload
    log(f"[bench] generating workload {wl}: {scenes.WORKLOAD_NAMES[wl]}")
    g_np, cams, opts = scenes.make_scene(wl)
    C_o, N = int(g_np["C_o"]), int(g_np["N"])
    Px = sum(c["W"] * c["H"] for c in cams)
    torch.cuda.set_device(0)
    if args.calibrate_copy:
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    copy_bw = measured_copy_bandwidth(torch)
    log(f"[bench] device-to-device copy of 1 GiB: {copy_bw / 1e9:.1f} GB/s (read + write)")
    hbm = lambda nbytes, sec: dict(achieved_gbps=round(nbytes / sec / 1e9, 1), peak_gbps=PEAK_HBM / 1e9,
                                   frac=round(nbytes / sec / PEAK_HBM, 4),
                                   frac_of_copy=round(nbytes / sec / copy_bw, 4))
    g = U.to_device(g_np)
    up = device_upstream(torch, Px, C_o, 1000 * wl)
    out = U.alloc_outputs(cams, C_o)
    grads = U.zeros_like_params(g)
    bf16 = bool(args.sem_bf16x3)
    rast = U.Rasterizer(prune_Tk=float(opts["prune_Tk"]), sem_bf16x3=int(bf16))
    if args.tile:
        tw, th = (int(x) for x in args.tile.split("x"))
        rast.set_options(tile_w=tw, tile_h=th, batch=args.batch)
    tuned = None
    if not args.no_autotune and not args.tile:
        log("[bench] autotuning tile shape and batch")
        tuned = rast.autotune(g, cams, out, up, grads, cache=False)  # always time here
        log(f"[bench] autotune -> {tuned}")

    # counters for the FLOP accounting (one eager forward) and the per-tile
    # workgroup times of the compositing kernels (one eager forward + backward)
    P = rast.project_and_sort(g, cams)
    rast.enable_counters(True)
    rast.forward(g, cams, out)
    F_eval, F_contrib = rast.read_counters()
    touched = rast.debug_buffer("touched")
    V_rec = int((touched > 0).sum().item())
    rast.backward(g, out, up, grads)
    torch.cuda.synchronize()
    balance, active = None, None
    if C_o > 8 and not (bf16 and C_o <= 32):
        balance = {k: tile_balance(rast.debug_buffer(b).cpu().numpy())
                   for k, b in (("render_fwd", "tile_clock_fwd"), ("render_bwd", "tile_clock_bwd"))}
        # (wavefront, list entry) pairs that the matrix-core backward walks
        bits = torch.tensor([bin(i).count("1") for i in range(256)], device="cuda", dtype=torch.int64)
        active = int(bits[rast.debug_buffer("activity_mask").view(torch.uint8).long()].sum().item())
    rast.enable_counters(False)
    log(f"[bench] pairs P={P} visible records={V_rec} evaluated={F_eval} contributing={F_contrib} "
        f"active wavefront entries={active}")
    log(f"[bench] tile balance {balance}")

    # per-stage durations (one eager step each) to find the dominant kernel
    ev = HipEvents()
    e0, e1 = ev.create(), ev.create()
    stage_ms = {}
    for st in STAGES:
        rast.time_stage(st, e0.value, e1.value)
        for t in grads.values():
            t.zero_()
        rast.forward(g, cams, out)
        rast.backward(g, out, up, grads)
        torch.cuda.synchronize()
        stage_ms[st] = ev.ms(e0, e1)
    dominant = max(stage_ms, key=stage_ms.get)
    log(f"[bench] stage ms {json.dumps({k: round(v, 3) for k, v in stage_ms.items()})} dominant={dominant}")

    # batched form: one captured graph per step; the dominant stage is bracketed
    # by HIP events recorded inside the graph, on the launch stream
    rast.time_stage(dominant, e0.value, e1.value)
    rast.capture_step(g, cams, out, up, grads)
    for _ in range(args.warmup):
        rast.replay()
    torch.cuda.synchronize()
    kern, steps_ev = [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        rast.replay()
        b.record()
        steps_ev.append((a, b))
        ev.sync(e1)
        kern.append(ev.ms(e0, e1))
    torch.cuda.synchronize()
    t_batched = (time.perf_counter() - t0) / args.steps
    step_list = [a.elapsed_time(b) for a, b in steps_ev]
    rast.time_stage(0)
    log(f"[bench] batched {t_batched * 1e3:.3f} ms/step (events median {pct(step_list, 50):.3f})  "
        f"{dominant} {np.median(kern):.3f} ms")

    t_pv = None
    if not args.no_per_view:
        t_pv = per_view_rate(torch, U, g, cams, out, up, grads, opts, rast.opts, C_o, args.steps, args.warmup, bf16)
        log(f"[bench] per-view {t_pv:.3f} ms/step")

    # forward-only form (viewer / inference): one captured graph per frame set,
    # no upstream, no gradients, no T_final / n_contrib stores
    fwd_only = None
    if not args.no_forward_only:
        fo = U.Rasterizer(prune_Tk=float(opts["prune_Tk"]), tile_w=rast.opts.tile_w, tile_h=rast.opts.tile_h,
                          batch=rast.opts.batch, sem_bf16x3=int(bf16))
        out_fo = U.alloc_outputs(cams, C_o, state=False)
        fo.capture_step(g, cams, out_fo, None, None)
        t_fo, _ = time_replays(torch, fo, args.steps, args.warmup)
        fwd_only = dict(value=round(Px / t_fo / 1e3, 2), unit="MP/s", ms_per_step=round(t_fo, 3),
                        views_per_s=round(len(cams) / t_fo * 1e3, 1))
        del fo, out_fo
        fh = U.Rasterizer(prune_Tk=float(opts["prune_Tk"]), tile_w=rast.opts.tile_w, tile_h=rast.opts.tile_h,
                          batch=rast.opts.batch, half_outputs=1, sem_bf16x3=int(bf16))
        out_h = U.alloc_outputs(cams, C_o, state=False, half=True)
        fh.capture_step(g, cams, out_h, None, None)
        fwd_only["half_outputs_ms_per_step"] = round(time_replays(torch, fh, args.steps, args.warmup)[0], 3)
        del fh, out_h
        log(f"[bench] forward-only {fwd_only}")

    # depth variants (the module ablation's ray-casting vs centre-point depth)
    depth_modes = None
    if not args.no_depth_modes:
        depth_modes = {"midpoint": round(t_batched * 1e3, 3)}
        for name, mode in (("centre", 1), ("hit_else_centre", 2)):
            dm = U.Rasterizer(prune_Tk=float(opts["prune_Tk"]), tile_w=rast.opts.tile_w, tile_h=rast.opts.tile_h,
                              batch=rast.opts.batch, depth_mode=mode, sem_bf16x3=int(bf16))
            out_dm = U.alloc_outputs(cams, C_o)
            dm.capture_step(g, cams, out_dm, up, grads)
            depth_modes[name] = round(time_replays(torch, dm, args.steps, args.warmup)[0], 3)
            del dm, out_dm
        depth_modes["unit"] = "ms per batched step"
        log(f"[bench] depth modes {depth_modes}")

    # differentiable pruning (section 3.3) with two optimiser-moment sets
    prune_res = None
    if not args.no_prune:
        moments = [{k: torch.zeros_like(g[k]) for k in U.PARAM_KEYS} for _ in range(2)]
        for _ in range(2):
            U.prune(g, 0.2, reset_k=True, states=moments)
        torch.cuda.synchronize()
        reps = 5
        t0 = time.perf_counter()
        for _ in range(reps):
            _, _, n_kept = U.prune(g, 0.2, reset_k=True, states=moments)
        torch.cuda.synchronize()
        t_pr = (time.perf_counter() - t0) / reps
        floats = sum(int(g[k].numel()) for k in U.PARAM_KEYS) // N
        b_pr = 3 * 4 * floats * (N + n_kept) + 4 * N
        prune_res = dict(ms=round(t_pr * 1e3, 3), kept=int(n_kept), gaussians=N, state_sets=2, **hbm(b_pr, t_pr),
                         note="includes the host read-back of the count")
        log(f"[bench] prune {prune_res}")
        del moments

    # training loss of section 3.4 on the batched outputs against synthetic targets
    loss_res = None
    if not args.no_loss:
        gen = torch.Generator(device="cuda").manual_seed(1000 * wl + 7)
        gt = dict(rgb=(out["rgb"] + 0.05 * torch.randn(out["rgb"].shape, device="cuda", generator=gen)).clamp_(0, 1),
                  depth=out["depth"] * (1 + 0.05 * torch.randn(out["depth"].shape, device="cuda", generator=gen)),
                  normal=torch.nn.functional.normalize(
                      out["normal"].view(-1, 3, 1) + 0.2 * torch.randn(out["normal"].numel() // 3, 3, 1,
                                                                       device="cuda", generator=gen), dim=1).view(-1),
                  label=torch.randint(0, max(C_o, 1), (Px,), device="cuda", generator=gen, dtype=torch.int32)
                  if C_o else None)
        reps = 10
        s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        times, values = {}, None
        for key, fuse in (("ms", False), ("fused_seeds_ms", True)):
            lossf = U.Loss(cams, C_o, fuse_normal=fuse, fuse_seg=fuse)
            for _ in range(2):
                lossf(out, gt)
            torch.cuda.synchronize()
            s0.record()
            for _ in range(reps):
                lv, _ = lossf(out, gt)
            s1.record()
            torch.cuda.synchronize()
            times[key] = s0.elapsed_time(s1) / reps
            if not fuse:
                values = dict(zip(U.LOSS_NAMES, [float(f"{float(x):.6g}") for x in lv.cpu()]))
            del lossf
        b_l = (96 + 8 * C_o) * Px  # every input map read once, every gradient map written once
        loss_res = dict(ms=round(times["ms"], 3), fused_seeds_ms=round(times["fused_seeds_ms"], 3), alg_bytes=int(b_l),
                        **hbm(b_l, times["ms"] * 1e-3), values=values)
        log(f"[bench] loss {loss_res}")
        del gt

    b_alg, f_fwd, f_bwd = algorithmic(N, V_rec, P, Px, C_o, int(g_np["sh_deg"]), F_eval, F_contrib)
    tiles = sum(-(-c["W"] // rast.opts.tile_w) * -(-c["H"] // rast.opts.tile_h) for c in cams)
    bs_bytes, bs_passes = binsort_bytes(V_rec, P, tiles)
    bs_ms = stage_ms["bin_sort"]
    bin_sort = dict(ms=round(bs_ms, 3), alg_bytes=int(bs_bytes), tile_sort_passes=bs_passes,
                    **hbm(bs_bytes, bs_ms * 1e-3))
    log(f"[bench] bin_sort {bin_sort}")
    k_ms = float(np.mean(kern))
    fl = None
    if dominant in ("render_bwd", "render_fwd"):
        fl = f_bwd if dominant == "render_bwd" else f_fwd
        achieved = fl / (k_ms * 1e-3) / 1e12
        roof = dict(bound="alu", achieved=round(achieved, 3), peak=PEAK_FP32 / 1e12, unit="TFLOP/s",
                    frac=round(achieved * 1e12 / PEAK_FP32, 4))
    else:
        achieved = b_alg / (k_ms * 1e-3) / 1e9
        roof = dict(bound="hbm", achieved=round(achieved, 1), peak=PEAK_HBM / 1e9, unit="GB/s",
                    frac=round(achieved * 1e9 / PEAK_HBM, 4))
    tr = profile_entry("traffic.json", dominant, wl)
    co = profile_entry("counters.json", dominant, wl)
    roof.update(kernel=dominant, launches=stage_launches(dominant, C_o, bf16),
                ms=round(k_ms, 4), ms_median=round(float(np.median(kern)), 4),
                traffic=None if tr is None else tr.get("bytes_per_launch"),
                counters=None if co is None else {k: round(v, 4) for k, v in co["derived"].items()},
                flops_per_launch=None if fl is None else float(fl))

    res = dict(metric=METRIC, value=round(Px / t_batched / 1e6, 2), unit="MP/s", n_gpus=1, steps=args.steps,
               warmup=args.warmup, ms_per_step=round(t_batched * 1e3, 3), higher_is_better=True, scaling="weak",
               vs_baseline=None, dtype="bf16x3" if (bf16 and 8 < C_o <= 32) else "f32", data="synthetic",
               config=dict(workload=scenes.WORKLOAD_NAMES[wl], gaussians=N, views=len(cams),
                           megapixels=round(Px / 1e6, 3), sh_degree=int(g_np["sh_deg"]), channels=C_o,
                           form="batched (one HIP graph per step)",
                           tile=f"{rast.opts.tile_w}x{rast.opts.tile_h}", batch=int(rast.opts.batch),
                           autotuned=tuned is not None),
               step_ms=dict(median=round(pct(step_list, 50), 3), p10=round(pct(step_list, 10), 3),
                            p90=round(pct(step_list, 90), 3)),
               per_view=None if t_pv is None else dict(value=round(Px / t_pv / 1e3, 2), unit="MP/s",
                                                        ms_per_step=round(t_pv, 3)),
               forward_only=fwd_only, prune=prune_res, loss=loss_res, depth_modes=depth_modes,
               step_hbm=dict(alg_bytes=int(b_alg), **hbm(b_alg, t_batched)),
               copy_gbps=round(copy_bw / 1e9, 1),
               bin_sort=bin_sort,
               counts=dict(pairs=P, records=V_rec, evaluated=F_eval, contributing=F_contrib,
                           active_wavefront_entries=active),
               tile_balance=balance,
               stage_ms={k: round(v, 4) for k, v in stage_ms.items()},
               roofline=roof, parity=None, cpu_baseline=None, secondary=None)
    if not args.no_cpu_baseline:
        log("[bench] timing the FP64 oracle on a sample and checking parity there")
        try:
            res["cpu_baseline"], res["parity"] = cpu_baseline(torch, U, g_np, cams, opts, rast, out)
            log(f"[bench] parity {res['parity']}")
        except Exception as ex:
            log(f"[bench] cpu baseline failed: {ex!r}")
    del rast, g, up, out, grads
    torch.cuda.empty_cache()
    if args.secondary and args.secondary != wl:
        log(f"[bench] secondary workload {args.secondary}")
        res["secondary"] = secondary_workload(torch, U, scenes, args.secondary, args.steps, args.warmup)
        log(f"[bench] secondary {res['secondary']}")
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
