"""Parity at the full workload sizes (the single-view 100k- and 500k-Gaussian
workloads and the two 16-view ones), in the launch configuration the benchmark
times (all views in one captured HIP graph, 16x16 tiles): the oracle evaluates
sampled pixels one by one (brute force over every Gaussian), and gradients are
checked with upstream weights that are non-zero only on those pixels."""
import numpy as np
import pytest

from tests import harness as Hn

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def O():
    from oracle import oracle
    oracle.lib()
    return oracle


def _sampled(O, workload, per_view, seed):
    import torch
    from paper_2510_12174_amd import scenes
    from paper_2510_12174_amd import unigs as U
    g, cams, opts = scenes.make_scene(workload)
    C_o = int(g["C_o"])
    Hn.say(f"[full w{workload}] N={g['N']} views={len(cams)} C_o={C_o}")
    rng = np.random.default_rng(seed)
    masks = []
    for cam in cams:
        m = np.zeros((cam["H"], cam["W"]), bool)
        m[rng.integers(4, cam["H"] - 4, per_view), rng.integers(4, cam["W"] - 4, per_view)] = True
        masks.append(m)
    # oracle forward at the sampled pixels (brute force per pixel)
    S = O._Scene(g)
    ora = [O.render(S, cam, opts, path=0, pixmask=m.astype(np.uint8)) for cam, m in zip(cams, masks)]
    # sparse upstream: N(0,1) weights on the sampled, unambiguous pixels only
    ups = []
    for cam, m, o in zip(cams, masks, ora):
        ok = m & (o["margin"] >= Hn.DELTA) & (o["grad_margin"] >= Hn.DELTA)
        H, W = cam["H"], cam["W"]
        u = dict(rgb=np.zeros((3, H, W), np.float32), depth=np.zeros((H, W), np.float32),
                 kmap=np.zeros((H, W), np.float32), normal=np.zeros((3, H, W), np.float32),
                 sem=np.zeros((C_o, H, W), np.float32))
        for k in ("rgb", "sem"):
            u[k][:, ok] = rng.standard_normal((u[k].shape[0], int(ok.sum()))).astype(np.float32)
        for k in ("depth", "kmap"):
            u[k][ok] = rng.standard_normal(int(ok.sum())).astype(np.float32)
        ups.append(u)
    # GPU: one captured step over all views
    gd = U.to_device(g)
    rast = U.Rasterizer(prune_Tk=float(opts["prune_Tk"]))
    out = U.alloc_outputs(cams, C_o)
    up = Hn.stack_upstream(ups, C_o)
    grads = U.zeros_like_params(gd)
    rast.capture_step(gd, cams, out, up, grads)
    rast.replay()
    rast.replay()
    torch.cuda.synchronize()
    outs = Hn.unstack(out, cams, C_o)
    gr = {k: grads[k].cpu().numpy().astype(np.float64) for k in Hn.PARAMS}
    return g, cams, opts, masks, ora, ups, outs, gr


@pytest.mark.timeout(600)
@pytest.mark.parametrize("workload,per_view", [(2, 96), (3, 96), (4, 24), (5, 12)])
def test_full_size_sampled(O, workload, per_view):
    g, cams, opts, masks, ora, ups, outs, gr = _sampled(O, workload, per_view, seed=31 + workload)
    worst = {}
    npx = 0
    for v, (cam, m, o, go) in enumerate(zip(cams, masks, ora, outs)):
        ok = m & (o["margin"] >= Hn.DELTA)
        npx += int(ok.sum())
        for k in ("rgb", "depth", "kmap", "sem", "T_final"):
            a, b = np.asarray(go[k], np.float64), o[k]
            d = np.abs(a - b)
            d = d[:, ok] if d.ndim == 3 else d[ok]
            worst[k] = max(worst.get(k, 0.0), float(d.max()) if d.size else 0.0)
        # normals stage-wise on the GPU's own depth
        on = O.normals(go["depth"], cam, opts, pixmask=m.astype(np.uint8))
        okn = m & (on["margin"] >= Hn.DELTA)
        dn = np.abs(go["normal"] - on["normal"])[:, okn]
        worst["normal(stage)"] = max(worst.get("normal(stage)", 0.0), float(dn.max()) if dn.size else 0.0)
    Hn.say(f"[full w{workload}] {npx} sampled pixels, max-abs {worst}")
    assert npx >= 0.8 * per_view * len(cams)
    for k, e in worst.items():
        assert e <= Hn.IMG_TOL, (k, e)
    # gradients from the sparse upstream
    ref = O.zero_grads(g)
    S = O._Scene(g)
    for cam, m, u, o in zip(cams, masks, ups, ora):
        O.backward(S, cam, u, o["depth"], opts, path=0, pixmask=m.astype(np.uint8), grads=ref)
    err = Hn.grad_errors(gr, ref, Hn.gauss_exclusions(O, g, cams, opts))
    Hn.say(f"[full w{workload}] grad err/tol {err}")
    for k, e in err.items():
        assert e <= 1.0, (k, e)


@pytest.mark.timeout(600)
def test_full_size_tile_lists_ordered():
    """The tile sort at full size (the 1M-Gaussian 16-view workload at 16 x 16
    tiles: 48,264 tiles, 16 bits in two passes over ~86M pairs, the first in
    full 8192-key LDS tiles): tile ids ascend; inside every tile's run the
    (FP32 camera-depth bits, index) pairs strictly increase, the order that
    section 3.4 fixes; each record's pairs number its emitted count; the ranges
    bracket the runs.  These hold at any size; the emitted set itself is
    checked against the plain definition at reduced sizes."""
    import torch
    from paper_2510_12174_amd import scenes
    from paper_2510_12174_amd import unigs as U
    g, cams, opts = scenes.make_scene(4)
    N, V = int(g["N"]), len(cams)
    rast = U.Rasterizer(tile_w=16, tile_h=16, prune_Tk=float(opts["prune_Tk"]))
    gd = U.to_device(g)
    P = rast.project_and_sort(gd, cams)
    torch.cuda.synchronize()
    keys = rast.debug_buffer("keys")[:P].view(torch.int32).to(torch.int64) & 0xFFFFFFFF
    vals = rast.debug_buffer("vals")[:P].view(torch.int32).to(torch.int64) & 0xFFFFFFFF
    ranges = rast.debug_buffer("ranges").view(torch.int32).to(torch.int64).reshape(-1, 2) & 0xFFFFFFFF
    rec = rast.debug_buffer("records").reshape(V * N, -1)
    touched = rast.debug_buffer("touched").view(torch.int32).to(torch.int64)
    ntiles = ranges.shape[0]
    Hn.say(f"[full w4 sort] pairs {P} tiles {ntiles}")
    assert ntiles > 1 << 15 and P > 4096 * 8192  # two passes, full first-pass tiles
    bases = torch.tensor([b for b in _tile_bases_16(cams)], device=keys.device, dtype=torch.int64)
    view = torch.searchsorted(bases, keys, right=True) - 1
    dbits = rec[view * N + vals, 7].contiguous().view(torch.int32).to(torch.int64) & 0xFFFFFFFF
    assert bool(torch.all(keys[1:] >= keys[:-1]))
    same = keys[1:] == keys[:-1]
    inc = (dbits[1:] > dbits[:-1]) | ((dbits[1:] == dbits[:-1]) & (vals[1:] > vals[:-1]))
    assert bool(torch.all(inc[same]))
    cnt = torch.bincount(view * N + vals, minlength=V * N)
    assert bool(torch.equal(cnt, touched[:V * N]))
    t = torch.arange(ntiles, device=keys.device, dtype=torch.int64)
    starts = torch.searchsorted(keys, t, right=False)
    ends = torch.searchsorted(keys, t, right=True)
    full = ends > starts
    assert bool(torch.equal(ranges[full, 0], starts[full])) and bool(torch.equal(ranges[full, 1], ends[full]))
    assert bool(torch.all(ranges[~full, 0] == ranges[~full, 1]))


def _tile_bases_16(cams):
    b, out = 0, []
    for c in cams:
        out.append(b)
        b += ((c["W"] + 15) // 16) * ((c["H"] + 15) // 16)
    return out
