#!/usr/bin/env python3
"""Benchmark: forward+backward megapixels/s of the multimodal Gaussian
rasterizer (RGB, ray-ellipsoid depth, normals, semantics, gradient factor), the
batched form (all views in one captured HIP graph) against the per-view form
(sequential per-view calls), on one MI355X.

Prints ONE JSON line.  `value` is the batched form's whole-job throughput with
all inputs resident in HBM; `per_view` carries the per-view form; `roofline`
reports the dominant kernel (timed live with HIP events on the launch stream)
against its roofline; `cpu_baseline` is the FP64 oracle on a bounded sample of
the same workload on the host cores.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload 4]
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
PEAK_FP32 = 157.3e12   # MI355X FP32 vector, FLOP/s
PEAK_HBM = 8.0e12      # MI355X HBM3E, B/s
STAGES = ["project", "bin_sort", "render_fwd", "normal_fwd", "normal_bwd", "render_bwd", "project_bwd"]
KERNEL_SOURCE = {"project": "project.hip", "bin_sort": "binsort.hip", "render_fwd": "render.hip",
                 "normal_fwd": "normal.hip", "normal_bwd": "normal.hip", "render_bwd": "render.hip",
                 "project_bwd": "project.hip"}


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


def algorithmic(N, V_rec, P, Px, C_o, sh_deg, F_eval, F_contrib):
    """Compulsory HBM bytes of one fwd+bwd step and per-kernel FLOPs."""
    S_h = 3 * (sh_deg + 1) ** 2
    Bp = 4 * N * (11 + S_h + C_o + 1)
    b = (3 * Bp + 64 * V_rec * 2 + 64 * V_rec * 2 + 44 * P + Px * (4 * (8 + C_o) + 8) + Px * 4 * (8 + C_o)
         + Px * 24)
    f_fwd = 12 * F_eval + F_contrib * (2 * (C_o + 5) + 24)
    f_bwd = 12 * F_eval + F_contrib * (4 * (C_o + 5) + 80)
    return b, f_fwd, f_bwd


def source_sha(name):
    p = os.path.join(ROOT, "paper_2510_12174_amd", "csrc", KERNEL_SOURCE[name])
    return hashlib.sha256(open(p, "rb").read()).hexdigest()[:16]


def traffic_for(name, workload, launches_per_step):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source (null otherwise)."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    d = json.load(open(p)).get(f"{name}@w{workload}")
    if not d or d.get("source_sha") != source_sha(name):
        return None
    return d.get("bytes_per_launch")


def valu_fraction_for(name, workload):
    """VALU issue fraction of the kernel (SQ_INSTS_VALU x 4 cycles over the
    SIMD cycles) from the committed counter summary, if taken on the current
    kernel source (null otherwise)."""
    p = os.path.join(ROOT, "profiles", "valu.json")
    if not os.path.exists(p):
        return None
    d = json.load(open(p)).get(f"{name}@w{workload}")
    if not d or d.get("source_sha") != source_sha(name):
        return None
    v = d.get("valu_issue_fraction")
    return None if v is None else round(v, 4)


def cpu_baseline(g, cams, opts, budget_s=15.0):
    """FP64 oracle (forward + normals + backward) on a bounded sample of the
    workload: whole views in order, then a band of central rows of the next
    view, sized from a short calibration run to about budget_s seconds."""
    from oracle import oracle as O
    from paper_2510_12174_amd import scenes
    S = O._Scene(g)

    def run(v, rows):
        cam = cams[v]
        H, W = cam["H"], cam["W"]
        ups = scenes.upstream([cam], g["C_o"], seed=4242 + v)
        pm = np.zeros((H, W), np.uint8)
        r0 = H // 2 - rows // 2
        pm[r0:r0 + rows] = 1
        t = time.perf_counter()
        o = O.render(S, cam, opts, path=1, pixmask=pm)
        O.normals(o["depth"], cam, opts, pixmask=pm)
        up = {k: (np.where(pm[None] > 0, u, 0) if u.ndim == 3 else np.where(pm > 0, u, 0))
              for k, u in ups[0].items()}
        O.backward(S, cam, up, o["depth"], opts, path=1, pixmask=pm)
        return time.perf_counter() - t, int(pm.sum())

    # calibration on view 0: fixed cost per view call and cost per pixel
    t1, p1 = run(0, 8)
    t2, p2 = run(0, 40)
    per_px = max((t2 - t1) / max(p2 - p1, 1), 1e-9)
    fixed = max(t1 - p1 * per_px, 0.0)
    total_t, total_px, parts, left = 0.0, 0, [], budget_s
    for v, cam in enumerate(cams):
        H, W = cam["H"], cam["W"]
        rows = int(min(H, max(4, (left - fixed) / (per_px * W))))
        t, px = run(v, rows)
        total_t += t
        total_px += px
        parts.append(f"view {v} ({W}x{H}) {'all' if rows == H else f'{rows} central'} rows")
        left -= t
        if rows < H or left <= fixed:
            break
    return dict(value=total_px / total_t / 1e6, unit="MP/s", cores=O.max_threads(), kind="oracle",
                sample=f"{', '.join(parts)} = {total_px} pixels, fwd+normals+bwd, {total_t:.1f} s")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", type=int, default=4)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-per-view", action="store_true")
    ap.add_argument("--no-forward-only", action="store_true")
    ap.add_argument("--no-prune", action="store_true")
    ap.add_argument("--no-loss", action="store_true")
    ap.add_argument("--no-depth-modes", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--tile", default=None, help="force a tile shape, e.g. 16x16")
    ap.add_argument("--batch", type=int, default=0, help="force the LDS batch (with --tile)")
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
    ups = scenes.upstream(cams, C_o, seed=1000 * wl)
    torch.cuda.set_device(0)
    if args.calibrate_copy:
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    g = U.to_device(g_np)
    cat = lambda k: torch.from_numpy(np.concatenate([u[k].reshape(-1) for u in ups])).cuda()
    up = dict(rgb=cat("rgb"), depth=cat("depth"), kmap=cat("kmap"), normal=cat("normal"),
              sem=cat("sem") if C_o else None)
    del ups
    out = U.alloc_outputs(cams, C_o)
    grads = U.zeros_like_params(g)
    rast = U.Rasterizer(prune_Tk=float(opts["prune_Tk"]))
    if args.tile:
        tw, th = (int(x) for x in args.tile.split("x"))
        rast.set_options(tile_w=tw, tile_h=th, batch=args.batch)
    tuned = None
    if not args.no_autotune and not args.tile:
        log("[bench] autotuning tile shape and batch")
        tuned = rast.autotune(g, cams, out, up, grads, cache=False)  # always time here
        log(f"[bench] autotune -> {tuned}")

    # counters for the FLOP accounting (one eager forward)
    P = rast.project_and_sort(g, cams)
    rast.enable_counters(True)
    rast.forward(g, cams, out)
    F_eval, F_contrib = rast.read_counters()
    rast.enable_counters(False)
    touched = rast.debug_buffer("touched")
    V_rec = int((touched > 0).sum().item())
    log(f"[bench] pairs P={P} visible records={V_rec} evaluated={F_eval} contributing={F_contrib}")

    # per-stage durations (one eager step each) to find the dominant kernel
    ev = HipEvents()
    e0, e1 = ev.create(), ev.create()
    stage_ms = {}
    for st in STAGES:
        rast.time_stage(st, e0.value, e1.value)
        grads_z = {k: v.zero_() for k, v in grads.items()}
        rast.forward(g, cams, out)
        rast.backward(g, out, up, grads_z)
        torch.cuda.synchronize()
        stage_ms[st] = ev.ms(e0, e1)
    dominant = max(stage_ms, key=stage_ms.get)
    log(f"[bench] stage ms {json.dumps({k: round(v, 3) for k, v in stage_ms.items()})} dominant={dominant}")

    # batched form: one captured graph per step, dominant kernel timed inside it
    rast.time_stage(dominant, e0.value, e1.value)
    rast.capture_step(g, cams, out, up, grads)
    for _ in range(args.warmup):
        rast.replay()
    torch.cuda.synchronize()
    kern = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        rast.replay()
        ev.sync(e1)
        kern.append(ev.ms(e0, e1))
    torch.cuda.synchronize()
    t_batched = (time.perf_counter() - t0) / args.steps
    rast.time_stage(0)
    log(f"[bench] batched {t_batched * 1e3:.3f} ms/step  {dominant} {np.mean(kern):.3f} ms")

    # per-view form: V sequential project -> bin_sort (pair count read back) ->
    # render_fwd -> render_bwd calls
    t_pv = None
    if not args.no_per_view:
        pr = U.Rasterizer(prune_Tk=float(opts["prune_Tk"]), tile_w=rast.opts.tile_w, tile_h=rast.opts.tile_h,
                          batch=rast.opts.batch)
        off = U.pixel_offsets(cams)
        views = []
        for v, cam in enumerate(cams):
            a, b = off[v], off[v + 1]
            sl = lambda t, c: None if t is None else t[c * a:c * b]
            views.append(([cam], {k: sl(out[k], c) for k, c in (("rgb", 3), ("depth", 1), ("kmap", 1),
                                                                ("normal", 3), ("sem", C_o), ("T_final", 1),
                                                                ("n_contrib", 1))},
                          {k: sl(up[k], c) for k, c in (("rgb", 3), ("depth", 1), ("kmap", 1), ("normal", 3),
                                                        ("sem", C_o))}))

        def per_view_step():
            for v in grads.values():
                v.zero_()
            for cv, ov, uv in views:
                pr.forward(g, cv, ov)
                pr.backward(g, ov, uv, grads)

        for _ in range(max(1, args.warmup)):
            per_view_step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            per_view_step()
        torch.cuda.synchronize()
        t_pv = (time.perf_counter() - t0) / args.steps
        log(f"[bench] per-view {t_pv * 1e3:.3f} ms/step")

    # forward-only form (viewer / inference): one captured graph per frame set,
    # no upstream, no gradients, no T_final / n_contrib stores
    fwd_only = None
    if not args.no_forward_only:
        fo = U.Rasterizer(prune_Tk=float(opts["prune_Tk"]), tile_w=rast.opts.tile_w, tile_h=rast.opts.tile_h,
                          batch=rast.opts.batch)
        out_fo = U.alloc_outputs(cams, C_o, state=False)
        fo.capture_step(g, cams, out_fo, None, None)
        for _ in range(args.warmup):
            fo.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            fo.replay()
        torch.cuda.synchronize()
        t_fo = (time.perf_counter() - t0) / args.steps
        fwd_only = dict(value=round(Px / t_fo / 1e6, 2), unit="MP/s", ms_per_step=round(t_fo * 1e3, 3),
                        views_per_s=round(len(cams) / t_fo, 1))
        # the same step writing binary16 colour, K, normal and semantic maps
        fh = U.Rasterizer(prune_Tk=float(opts["prune_Tk"]), tile_w=rast.opts.tile_w, tile_h=rast.opts.tile_h,
                          batch=rast.opts.batch, half_outputs=1)
        out_h = U.alloc_outputs(cams, C_o, state=False, half=True)
        fh.capture_step(g, cams, out_h, None, None)
        for _ in range(args.warmup):
            fh.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            fh.replay()
        torch.cuda.synchronize()
        fwd_only["half_outputs_ms_per_step"] = round((time.perf_counter() - t0) / args.steps * 1e3, 3)
        del fh, out_h
        log(f"[bench] forward-only {t_fo * 1e3:.3f} ms per {len(cams)} views ({fwd_only['value']} MP/s)")
        del fo, out_fo

    # depth variants (the module ablation's ray-casting vs centre-point depth):
    # the same batched step with depth_mode 1 (centre) and 2 (midpoint where the
    # ray meets the ellipsoid, centre elsewhere)
    depth_modes = None
    if not args.no_depth_modes:
        depth_modes = {"midpoint": round(t_batched * 1e3, 3)}
        for name, mode in (("centre", 1), ("hit_else_centre", 2)):
            dm = U.Rasterizer(prune_Tk=float(opts["prune_Tk"]), tile_w=rast.opts.tile_w, tile_h=rast.opts.tile_h,
                              batch=rast.opts.batch, depth_mode=mode)
            out_dm = U.alloc_outputs(cams, C_o)
            dm.capture_step(g, cams, out_dm, up, grads)
            for _ in range(args.warmup):
                dm.replay()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                dm.replay()
            torch.cuda.synchronize()
            depth_modes[name] = round((time.perf_counter() - t0) / args.steps * 1e3, 3)
            del dm, out_dm
        depth_modes["unit"] = "ms per batched step"
        log(f"[bench] depth modes {depth_modes}")

    # differentiable pruning (section 3.3): compaction of the parameters and two
    # optimiser-moment sets at T_k = 0.2; HBM-bound (every array read once, the
    # kept part written once)
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
        floats = sum(int(g[k].numel()) for k in U.PARAM_KEYS) // N  # per Gaussian
        b_pr = 3 * 4 * floats * (N + n_kept) + 4 * N
        prune_res = dict(ms=round(t_pr * 1e3, 3), kept=int(n_kept), gaussians=N, state_sets=2,
                         achieved_gbps=round(b_pr / t_pr / 1e9, 1), peak_gbps=PEAK_HBM / 1e9,
                         frac=round(b_pr / t_pr / PEAK_HBM, 4), note="includes the host read-back of the count")
        log(f"[bench] prune {prune_res}")
        del moments

    # training loss of section 3.4 on the batched outputs against synthetic
    # targets: values and every upstream map, on the device (graph-capturable)
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
        lossf = U.Loss(cams, C_o)
        for _ in range(2):
            lossf(out, gt)
        torch.cuda.synchronize()
        reps = 10
        s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s0.record()
        for _ in range(reps):
            lv, _ = lossf(out, gt)
        s1.record()
        torch.cuda.synchronize()
        t_l = s0.elapsed_time(s1) / reps * 1e-3
        b_l = (96 + 8 * C_o) * Px  # every input map read once, every gradient map written once
        # the same loss with the cosine and cross-entropy seeds left to the
        # backward (no normal or semantic gradient maps written)
        lossx = U.Loss(cams, C_o, fuse_normal=True, fuse_seg=True)
        for _ in range(2):
            lossx(out, gt)
        torch.cuda.synchronize()
        s0.record()
        for _ in range(reps):
            lossx(out, gt)
        s1.record()
        torch.cuda.synchronize()
        t_lx = s0.elapsed_time(s1) / reps * 1e-3
        loss_res = dict(ms=round(t_l * 1e3, 3), fused_seeds_ms=round(t_lx * 1e3, 3), alg_bytes=int(b_l),
                        achieved_gbps=round(b_l / t_l / 1e9, 1),
                        peak_gbps=PEAK_HBM / 1e9, frac=round(b_l / t_l / PEAK_HBM, 4),
                        values=dict(zip(U.LOSS_NAMES, [float(f"{float(x):.6g}") for x in lv.cpu()])))
        log(f"[bench] loss {loss_res}")
        del gt, lossf, lossx

    # quick parity spot check of the timed batched outputs (view 0, sampled pixels)
    parity = None
    try:
        from oracle import oracle as O
        rast.replay()
        torch.cuda.synchronize()
        cam = cams[0]
        rng = np.random.default_rng(7)
        pm = np.zeros((cam["H"], cam["W"]), np.uint8)
        pm[rng.integers(0, cam["H"], 48), rng.integers(0, cam["W"], 48)] = 1
        o = O.render(g_np, cam, opts, path=0, pixmask=pm)
        sel = (pm > 0) & (o["margin"] >= 1e-5)
        Pv = cam["W"] * cam["H"]
        gd = out["depth"][:Pv].cpu().numpy().reshape(cam["H"], cam["W"])
        grgb = out["rgb"][:3 * Pv].cpu().numpy().reshape(3, cam["H"], cam["W"])
        gs = out["sem"][:C_o * Pv].cpu().numpy().reshape(C_o, cam["H"], cam["W"]) if C_o else None
        e = max(float(np.abs(gd - o["depth"])[sel].max()), float(np.abs(grgb - o["rgb"])[:, sel].max()),
                float(np.abs(gs - o["sem"])[:, sel].max()) if C_o else 0.0)
        parity = dict(pixels=int(sel.sum()), max_abs=e, tol=1e-4, ok=bool(e <= 1e-4))
        log(f"[bench] parity spot check {parity}")
    except Exception as ex:  # the oracle is optional on a bare box
        log(f"[bench] parity spot check skipped: {ex}")

    b_alg, f_fwd, f_bwd = algorithmic(N, V_rec, P, Px, C_o, int(g_np["sh_deg"]), F_eval, F_contrib)
    k_ms = float(np.mean(kern))
    if dominant in ("render_bwd", "render_fwd"):
        fl = f_bwd if dominant == "render_bwd" else f_fwd
        achieved = fl / (k_ms * 1e-3) / 1e12
        roof = dict(bound="alu", achieved=round(achieved, 3), peak=PEAK_FP32 / 1e12, unit="TFLOP/s",
                    frac=round(achieved * 1e12 / PEAK_FP32, 4))
    else:
        # streaming kernels: bytes of the stage's own compulsory traffic are not
        # separated here; report the step's compulsory bytes over the stage time
        achieved = b_alg / (k_ms * 1e-3) / 1e9
        roof = dict(bound="hbm", achieved=round(achieved, 1), peak=PEAK_HBM / 1e9, unit="GB/s",
                    frac=round(achieved * 1e9 / PEAK_HBM, 4))
    roof.update(kernel=dominant, ms=round(k_ms, 4), traffic=traffic_for(dominant, wl, 1),
                valu_issue=valu_fraction_for(dominant, wl))

    res = dict(metric=METRIC, value=round(Px / t_batched / 1e6, 2), unit="MP/s", n_gpus=1, steps=args.steps,
               warmup=args.warmup, ms_per_step=round(t_batched * 1e3, 3), higher_is_better=True, scaling="weak",
               vs_baseline=None, dtype="f32", data="synthetic",
               config=dict(workload=scenes.WORKLOAD_NAMES[wl], gaussians=N, views=len(cams),
                           megapixels=round(Px / 1e6, 3), sh_degree=int(g_np["sh_deg"]), channels=C_o,
                           form="batched (one HIP graph per step)",
                           tile=f"{rast.opts.tile_w}x{rast.opts.tile_h}", batch=int(rast.opts.batch),
                           autotuned=tuned is not None),
               per_view=None if t_pv is None else dict(value=round(Px / t_pv / 1e6, 2), unit="MP/s",
                                                        ms_per_step=round(t_pv * 1e3, 3)),
               forward_only=fwd_only, prune=prune_res, loss=loss_res, depth_modes=depth_modes,
               step_hbm=dict(alg_bytes=int(b_alg), frac=round(b_alg / t_batched / PEAK_HBM, 4)),
               counts=dict(pairs=P, records=V_rec, evaluated=F_eval, contributing=F_contrib),
               stage_ms={k: round(v, 4) for k, v in stage_ms.items()},
               roofline=roof, parity=parity, cpu_baseline=None)
    if not args.no_cpu_baseline:
        log("[bench] timing the FP64 oracle on a sample")
        try:
            res["cpu_baseline"] = cpu_baseline(g_np, cams, opts)
        except Exception as ex:
            log(f"[bench] cpu baseline failed: {ex}")
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
