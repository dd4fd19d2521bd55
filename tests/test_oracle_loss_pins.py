"""Pins of the FP64 loss reference (section 3.4) against facts fixed outside it:
brute-force window sums, a library Gaussian filter, SSIM's closed forms,
cross-entropy identities and finite differences of the total loss."""
import math

import numpy as np
import pytest
from scipy.ndimage import gaussian_filter
from scipy.special import logsumexp

from oracle import loss as L


def _rng(s):
    return np.random.default_rng(s)


def test_window_sum_matches_pixel_loop():
    """Per-pixel double loop over in-image neighbours (a different route than
    the shifted-array sum) on an image smaller than the window."""
    x = _rng(0).normal(size=(7, 9))
    w1 = np.exp(-np.arange(-5, 6) ** 2 / (2 * 1.5 ** 2))
    w1 /= w1.sum()
    H, W = x.shape
    ref = np.zeros_like(x)
    for v in range(H):
        for u in range(W):
            for yy in range(H):
                for xx in range(W):
                    if abs(yy - v) <= 5 and abs(xx - u) <= 5:
                        ref[v, u] += w1[yy - v + 5] * w1[xx - u + 5] * x[yy, xx]
    np.testing.assert_allclose(L.window_sum(x), ref, rtol=0, atol=1e-14)


def test_window_sum_matches_library_gaussian_filter():
    """scipy's separable Gaussian filter with radius 5 and zero padding is the
    same operator."""
    x = _rng(1).random((40, 33))
    ref = gaussian_filter(x, sigma=1.5, mode="constant", cval=0.0, truncate=5 / 1.5)
    np.testing.assert_allclose(L.window_sum(x), ref, rtol=0, atol=1e-14)


def test_ssim_of_identical_images_is_one():
    x = _rng(2).random((20, 17))
    np.testing.assert_allclose(L.ssim_map(x, x), 1.0, atol=1e-12)


def test_ssim_of_constant_images_closed_form():
    """Away from the border (no zero padding inside the window) constants a, b
    have no variance: SSIM = (2ab + C1) / (a^2 + b^2 + C1)."""
    a, b = 0.3, 0.7
    S = L.ssim_map(np.full((24, 24), a), np.full((24, 24), b))
    ref = (2 * a * b + 1e-4) / (a * a + b * b + 1e-4)
    np.testing.assert_allclose(S[5:-5, 5:-5], ref, rtol=1e-11)  # moments cancel to ~1e-16
    assert abs(S[0, 0] - ref) > 1e-6  # the padded corner differs


def test_ssim_matches_library_filter_formula():
    """SSIM of Wang et al. from scipy-filtered moments."""
    r = _rng(3)
    x, y = r.random((30, 26)), r.random((30, 26))
    f = lambda a: gaussian_filter(a, sigma=1.5, mode="constant", truncate=5 / 1.5)
    mx, my = f(x), f(y)
    sxx, syy, sxy = f(x * x) - mx ** 2, f(y * y) - my ** 2, f(x * y) - mx * my
    ref = (2 * mx * my + 1e-4) * (2 * sxy + 9e-4) / ((mx ** 2 + my ** 2 + 1e-4) * (sxx + syy + 9e-4))
    np.testing.assert_allclose(L.ssim_map(x, y), ref, rtol=1e-12, atol=1e-13)


def test_ssim_gradient_matches_fd():
    r = _rng(4)
    x, y, gS = r.random((13, 12)), r.random((13, 12)), r.normal(size=(13, 12))
    g = L.ssim_grad(x, y, gS)
    h = 1e-6
    for (v, u) in [(0, 0), (6, 5), (12, 11), (3, 10), (12, 0)]:
        xp, xm = x.copy(), x.copy()
        xp[v, u] += h
        xm[v, u] -= h
        fd = ((gS * L.ssim_map(xp, y)).sum() - (gS * L.ssim_map(xm, y)).sum()) / (2 * h)
        assert abs(g[v, u] - fd) <= 1e-7 * max(1.0, abs(fd)), (v, u, g[v, u], fd)


def test_cross_entropy_identities():
    r = _rng(5)
    C, H, W = 7, 5, 6
    z = r.normal(size=(C, H, W)) * 3
    lab = r.integers(0, C, size=(H, W))
    lab[0, 0], lab[1, 1] = -1, C  # ignored pixels
    ce, g = L.cross_entropy(z, lab)
    ref = logsumexp(z, axis=0) - np.take_along_axis(z, np.clip(lab, 0, C - 1)[None], 0)[0]
    ok = (lab >= 0) & (lab < C)
    np.testing.assert_allclose(ce[ok], ref[ok], rtol=1e-13)
    assert ce[0, 0] == 0 and ce[1, 1] == 0 and np.all(g[:, 0, 0] == 0)
    np.testing.assert_allclose(g.sum(axis=0), 0.0, atol=1e-14)  # softmax minus one-hot
    u, _ = L.cross_entropy(np.zeros((C, 2, 2)), np.zeros((2, 2), int))
    np.testing.assert_allclose(u, math.log(C), rtol=1e-15)
    # finite differences of one pixel's cross-entropy
    h = 1e-6
    for c in range(C):
        zp, zm = z.copy(), z.copy()
        zp[c, 2, 3] += h
        zm[c, 2, 3] -= h
        fd = (L.cross_entropy(zp, lab)[0][2, 3] - L.cross_entropy(zm, lab)[0][2, 3]) / (2 * h)
        assert abs(g[c, 2, 3] - fd) < 1e-8


def _maps(seed, sizes, C_o=5, all_targets=True):
    r = _rng(seed)
    outs, gts = [], []
    for (W, H) in sizes:
        n = r.normal(size=(3, H, W))
        n /= np.linalg.norm(n, axis=0)
        ng = r.normal(size=(3, H, W))
        ng /= np.linalg.norm(ng, axis=0)
        outs.append(dict(rgb=r.random((3, H, W)), depth=r.uniform(0.5, 4, (H, W)), kmap=r.uniform(0.7, 1.2, (H, W)),
                         normal=n, sem=r.normal(size=(C_o, H, W)) * 2))
        t = dict(rgb=r.random((3, H, W)))
        if all_targets:
            t.update(depth=r.uniform(0.5, 4, (H, W)), normal=ng, label=r.integers(0, C_o, (H, W)))
        gts.append(t)
    return outs, gts


def test_total_loss_balanced_closed_form():
    """With every term positive the balanced total is L_l1 (lambda_1 + sum of
    the other lambdas)."""
    outs, gts = _maps(6, [(9, 8), (6, 11)])
    Lv, _ = L.total_loss(outs, gts)
    for k in ("l1", "ssim", "normal", "depth", "seg", "K"):
        assert Lv[k] > 0
    assert abs(Lv["all"] - Lv["l1"] * 1.5) < 1e-14
    Lu, _ = L.total_loss(outs, gts, balance=False)
    ref = Lu["l1"] + 0.1 * (Lu["ssim"] + Lu["normal"] + Lu["depth"] + Lu["seg"] + Lu["K"])
    assert abs(Lu["all"] - ref) < 1e-14


def test_normal_loss_extremes():
    outs, gts = _maps(7, [(5, 4)])
    gts[0]["normal"] = outs[0]["normal"].copy()
    assert abs(L.total_loss(outs, gts)[0]["normal"]) < 1e-14
    gts[0]["normal"] = -outs[0]["normal"]
    assert abs(L.total_loss(outs, gts)[0]["normal"] - 2.0) < 1e-14


@pytest.mark.parametrize("balance", [True, False])
def test_total_loss_gradient_matches_fd(balance):
    """Finite differences of L_all with the balancing ratios frozen at the
    point (they are constants in the gradient): the balanced total equals the
    unbalanced one with lambda_x w_x as weights."""
    outs, gts = _maps(8, [(14, 9), (7, 12)])
    Lv, g = L.total_loss(outs, gts, balance=balance)
    lam = np.array(L.DEFAULT_LAMBDAS)
    names = ("l1", "ssim", "normal", "depth", "seg", "K")
    if balance:
        lam = np.array([lam[0]] + [lam[k] * abs(Lv["l1"]) / abs(Lv[n]) for k, n in enumerate(names) if k > 0])
    frozen = lambda o: L.total_loss(o, gts, lambdas=lam, balance=False)[0]["all"]
    assert abs(frozen(outs) - Lv["all"]) < 1e-14
    h = 1e-6
    r = _rng(9)
    for key in ("rgb", "depth", "kmap", "normal", "sem"):
        for _ in range(4):
            v = int(r.integers(0, 2))
            a = outs[v][key]
            idx = tuple(int(r.integers(0, s)) for s in a.shape)
            op = [dict(o) for o in outs]
            om = [dict(o) for o in outs]
            op[v][key] = a.copy()
            om[v][key] = a.copy()
            op[v][key][idx] += h
            om[v][key][idx] -= h
            fd = (frozen(op) - frozen(om)) / (2 * h)
            assert abs(g[v][key][idx] - fd) <= 1e-8 + 1e-6 * abs(fd), (key, idx, g[v][key][idx], fd)


def test_missing_targets_drop_terms():
    outs, gts = _maps(10, [(8, 8)], all_targets=False)
    Lv, g = L.total_loss(outs, gts)
    assert Lv["normal"] == Lv["depth"] == Lv["seg"] == 0.0
    assert abs(Lv["all"] - Lv["l1"] * 1.2) < 1e-14  # lambda_1 + lambda_ssim + lambda_K
    assert not g[0]["depth"].any() and not g[0]["normal"].any() and not g[0]["sem"].any()
