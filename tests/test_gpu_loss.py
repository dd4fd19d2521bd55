"""The section-3.4 loss on the GPU (ugs_loss) against the FP64 reference:
loss values and every gradient map, on synthetic maps over ragged views (one
smaller than the SSIM window), on maps the rasterizer rendered, and on two
full-resolution views of the batched workload."""
import numpy as np
import pytest

from tests import harness as Hn

pytestmark = pytest.mark.gpu

LOSS_REL = 2e-5   # loss values: |L - L_ref| <= 2e-5 |L_ref| + 1e-6
NAMES = ("l1", "ssim", "normal", "depth", "seg", "K", "all", "ssim_mean")


def synth(seed, sizes, C_o, targets=True, bad_labels=True):
    r = np.random.default_rng(seed)
    outs, gts = [], []
    f32 = lambda a: np.ascontiguousarray(a, np.float32)
    for (W, H) in sizes:
        n = r.normal(size=(3, H, W))
        n /= np.linalg.norm(n, axis=0)
        ng = r.normal(size=(3, H, W))
        ng /= np.linalg.norm(ng, axis=0)
        outs.append(dict(rgb=f32(r.random((3, H, W))), depth=f32(r.uniform(0.5, 4, (H, W))),
                         kmap=f32(r.uniform(0.7, 1.2, (H, W))), normal=f32(n),
                         sem=f32(r.normal(size=(C_o, H, W)) * 2)))
        t = dict(rgb=f32(np.clip(outs[-1]["rgb"] + r.normal(size=(3, H, W)) * 0.1, 0, 1)))
        if targets:
            lab = r.integers(0, C_o, (H, W)).astype(np.int32)
            if bad_labels:
                lab[r.random((H, W)) < 0.02] = -1
                lab[r.random((H, W)) < 0.02] = C_o
            t.update(depth=f32(r.uniform(0.5, 4, (H, W))), normal=f32(ng), label=lab)
        gts.append(t)
    return outs, gts


def run_gpu(cams, C_o, outs, gts, balance=True):
    import torch
    from paper_2510_12174_amd import unigs as U
    cat = lambda key, lst: torch.from_numpy(np.concatenate([np.asarray(d[key]).reshape(-1) for d in lst])).cuda()
    out = {k: cat(k, outs) for k in ("rgb", "depth", "kmap", "normal", "sem")}
    gt = {k: (cat(k, gts) if gts[0].get(k) is not None else None) for k in ("rgb", "depth", "normal", "label")}
    loss = U.Loss(cams, C_o, balance=balance)
    losses, grad = loss(out, gt)
    torch.cuda.synchronize()
    Lv = dict(zip(U.LOSS_NAMES, losses.cpu().numpy().astype(np.float64)))
    gv = []
    views = {k: U.split_views(grad[k], cams, c) for k, c in (("rgb", 3), ("depth", 1), ("kmap", 1), ("normal", 3))}
    views["sem"] = U.split_views(grad["sem"], cams, C_o)
    for v, cam in enumerate(cams):
        d = {k: views[k][v].cpu().numpy().astype(np.float64) for k in views}
        for k in ("depth", "kmap"):
            d[k] = d[k].reshape(cam["H"], cam["W"])
        gv.append(d)
    return Lv, gv


def compare(cams, C_o, outs, gts, balance=True, tag=""):
    from oracle import loss as OL
    Lg, gg = run_gpu(cams, C_o, outs, gts, balance)
    Lr, gr = OL.total_loss(outs, gts, balance=balance)
    for k in NAMES:
        err = abs(Lg[k] - Lr[k])
        Hn.say(f"[loss {tag}] {k}: gpu {Lg[k]:.8g} ref {Lr[k]:.8g} err {err:.3g}")
        assert err <= LOSS_REL * abs(Lr[k]) + 1e-6, k
    # per-term gradient coefficients (d L_all / d map element), from the FP64 values
    P = sum(int(c["W"]) * int(c["H"]) for c in cams)
    lam = OL.DEFAULT_LAMBDAS
    on = dict(l1=True, ssim=True, normal=gts[0].get("normal") is not None, depth=gts[0].get("depth") is not None,
              seg=gts[0].get("label") is not None, K=True)
    for k, (n, sign, den) in enumerate([("l1", 1, 3), ("ssim", -1, 3), ("normal", -1, 1), ("depth", 1, 1),
                                        ("seg", 1, 1), ("K", 1, 1)]):
        w = 1.0 if (n == "l1" or not balance) else (abs(Lr["l1"]) / abs(Lr[n]) if Lr[n] != 0 else 0.0)
        ref = sign * lam[k] * (w if on[n] else 0.0) / (den * P)
        got = Lg["coef_" + n]
        assert abs(got - ref) <= LOSS_REL * abs(ref) + 1e-12, (n, got, ref)
    for key in ("rgb", "depth", "kmap", "normal", "sem"):
        a = np.concatenate([g[key].reshape(-1) for g in gg])
        b = np.concatenate([np.asarray(g[key], np.float64).reshape(-1) for g in gr])
        rms = float(np.sqrt(np.mean(b * b))) if b.size else 0.0
        e = float(np.max(np.abs(a - b) / (Hn.GRAD_REL * np.abs(b) + Hn.GRAD_REL * rms + 1e-30))) if b.size else 0.0
        Hn.say(f"[loss {tag}] grad {key}: rms {rms:.3g} err/tol {e:.3g}")
        assert e <= 1.0, key


def cams_of(sizes):
    return [dict(W=W, H=H, fx=100.0, fy=100.0, cx=W / 2, cy=H / 2, R=np.eye(3), t=np.zeros(3)) for W, H in sizes]


SIZES = [(96, 72), (120, 68), (130, 97), (5, 3)]   # ragged: one pixel per thread
SIZES4 = [(96, 72), (120, 68), (68, 20)]            # pixel counts divisible by 4: four per thread


@pytest.mark.parametrize("sizes,C_o,balance", [(SIZES, 12, True), (SIZES, 12, False), (SIZES4, 12, True),
                                               (SIZES4, 13, False), (SIZES, 1, True)])
def test_loss_matches_reference_synthetic(sizes, C_o, balance):
    outs, gts = synth(1, sizes, C_o)
    compare(cams_of(sizes), C_o, outs, gts, balance, f"synthetic {len(sizes)} views C_o={C_o} balance={balance}")


def test_loss_without_optional_targets():
    outs, gts = synth(2, SIZES[:2], 4, targets=False)
    compare(cams_of(SIZES[:2]), 4, outs, gts, True, "rgb only")


def test_loss_on_rendered_maps():
    """The rasterizer's own outputs (K near 1, logits of rendered channels,
    normals from depth) against targets of another seed's rendering."""
    g, cams, opts = Hn.small_workload("w4s")
    C_o = int(g["C_o"])
    outs, _, _ = Hn.gpu_run(g, cams, opts)
    g2, _, _ = Hn.small_workload("w4s", seed=1)
    tgt, _, _ = Hn.gpu_run(g2, cams, opts)
    gts = []
    for o, t in zip(outs, tgt):
        gts.append(dict(rgb=t["rgb"], depth=t["depth"], normal=t["normal"],
                        label=np.argmax(t["sem"], axis=0).astype(np.int32)))
    outs = [{k: np.ascontiguousarray(o[k], np.float32) for k in ("rgb", "depth", "kmap", "normal", "sem")}
            for o in outs]
    compare(cams, C_o, outs, gts, True, "rendered w4s")


def test_fused_cosine_seed_matches_map():
    """The cosine seed formed inside the normal backward (normal_target and the
    device coefficient losses[10]) gives the same parameter gradients as the
    loss's explicit normal-gradient map."""
    import torch
    from paper_2510_12174_amd import unigs as U
    g, cams, opts = Hn.small_workload("w4s")
    C_o = int(g["C_o"])
    gd = U.to_device(g)
    rast = U.Rasterizer()
    out = rast.forward(gd, cams)
    _, gts = synth(5, [(c["W"], c["H"]) for c in cams], C_o, bad_labels=False)
    cat = lambda key: torch.from_numpy(np.concatenate([np.asarray(d[key]).reshape(-1) for d in gts])).cuda()
    gt = {k: cat(k) for k in ("rgb", "depth", "normal", "label")}
    _, up_map = U.Loss(cams, C_o)(out, gt)
    _, up_fused = U.Loss(cams, C_o, fuse_normal=True)(out, gt)
    assert up_fused["normal"] is None and up_fused["normal_scale"].numel() == 1
    # G_D (depth upstream plus the normal branch, the normal backward's output)
    # is formed without atomics: bit-identical; the parameter gradients go
    # through float atomics, so they agree to rounding
    a = rast.backward(gd, out, up_map)
    gd_map = rast.debug_buffer("depth_grad").clone()
    rast.forward(gd, cams, out)  # one backward per projection
    b = rast.backward(gd, out, up_fused)
    gd_fused = rast.debug_buffer("depth_grad").clone()
    torch.cuda.synchronize()
    assert float(gd_map.abs().sum()) > 0 and torch.equal(gd_map, gd_fused)
    for k in U.PARAM_KEYS:
        x, y = a[k].cpu().numpy().astype(np.float64), b[k].cpu().numpy().astype(np.float64)
        if x.size:
            rms = np.sqrt(np.mean(x * x)) + 1e-30
            assert np.max(np.abs(x - y)) <= 1e-4 * rms, (k, np.max(np.abs(x - y)) / rms)
    Hn.say("[loss] fused cosine seed equals the explicit normal map")


def test_fused_cross_entropy_seed_matches_map():
    """The cross-entropy seed formed inside the render backward from the
    rendered logits, the labels and losses[12] gives the parameter gradients of
    the loss's explicit semantic-gradient map (to the rounding of the two
    log-sum-exp evaluations and float-atomic order); both forward kernels'
    backward forms run (32 channels on the matrix cores, 64 on the vector
    path)."""
    import torch
    from paper_2510_12174_amd import unigs as U
    for kind in ("w4s", "w3s"):
        g, cams, opts = Hn.small_workload(kind)
        C_o = int(g["C_o"])
        gd = U.to_device(g)
        rast = U.Rasterizer()
        out = rast.forward(gd, cams)
        _, gts = synth(6, [(c["W"], c["H"]) for c in cams], C_o)
        cat = lambda key: torch.from_numpy(np.concatenate([np.asarray(d[key]).reshape(-1) for d in gts])).cuda()
        gt = {k: cat(k) for k in ("rgb", "depth", "normal", "label")}
        _, up_map = U.Loss(cams, C_o)(out, gt)
        lf, up_fused = U.Loss(cams, C_o, fuse_normal=True, fuse_seg=True)(out, gt)
        assert up_fused["sem"] is None and up_fused["normal"] is None
        a = rast.backward(gd, out, up_map)
        rast.forward(gd, cams, out)  # one backward per projection
        b = rast.backward(gd, out, up_fused)
        torch.cuda.synchronize()
        for k in U.PARAM_KEYS:
            x, y = a[k].cpu().numpy().astype(np.float64), b[k].cpu().numpy().astype(np.float64)
            if x.size:
                rms = np.sqrt(np.mean(x * x)) + 1e-30
                err = np.max(np.abs(x - y)) / rms
                Hn.say(f"[loss {kind}] fused seeds vs maps, {k}: max err / rms {err:.2e}")
                assert err <= 1e-4, k


def test_loss_graph_capture_replays():
    """ugs_loss is asynchronous and allocation-free, so it can be captured in a
    graph: every replay on new map contents equals an eager call on them (the
    partial sums are added in a fixed order, so bit for bit)."""
    import torch
    from paper_2510_12174_amd import unigs as U
    sizes = SIZES4
    cams = cams_of(sizes)
    C_o = 12
    outs, gts = synth(7, sizes, C_o)
    cat = lambda key, lst: torch.from_numpy(np.concatenate([np.asarray(d[key]).reshape(-1) for d in lst])).cuda()
    out = {k: cat(k, outs) for k in ("rgb", "depth", "kmap", "normal", "sem")}
    gt = {k: cat(k, gts) for k in ("rgb", "depth", "normal", "label")}
    cap = U.Loss(cams, C_o)
    cap(out, gt)  # warm-up outside the capture
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        cap(out, gt)
    eager = U.Loss(cams, C_o)
    for rep in range(3):
        with torch.no_grad():
            out["rgb"].copy_(torch.rand_like(out["rgb"]))
            out["kmap"].mul_(1.01)
        graph.replay()
        torch.cuda.synchronize()
        _ = torch.ones(10, device="cuda").sum().item()
        lv, gv = eager(out, gt)
        torch.cuda.synchronize()
        assert torch.equal(cap.losses, lv), rep
        for k in ("rgb", "depth", "kmap", "normal", "sem"):
            assert torch.equal(cap.grad[k], gv[k]), (rep, k)


def test_loss_full_resolution_views():
    """Two views at the batched workload's 1200x680 and 1296x968 resolutions,
    32 channels, launched as in the benchmark (one launch per view and pass)."""
    sizes = [(1200, 680), (1296, 968)]
    outs, gts = synth(3, sizes, 32, bad_labels=False)
    compare(cams_of(sizes), 32, outs, gts, True, "full resolution")
