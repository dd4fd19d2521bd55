"""FP64 reference of the training loss of section 3.4 ("Loss Function") and of
its gradient with respect to the rendered maps.

TEST INFRASTRUCTURE ONLY: imported by tests/ and the benchmark's CPU-baseline
leg, never by the product package; it shares no code with the HIP path.

Inputs are per-view maps in the rasterizer's layouts ([3][H][W] colour and
normal, [H][W] depth and K, [C_o][H][W] logits) as float32 arrays, promoted to
float64 here.  Every term is a mean over the P pixels of all views (colour
terms over the 3P colour values):
  L_l1     mean |C - C_gt|                                   (section 3.4)
  L_ssim   1 - mean SSIM per colour channel                  (section 3.4; SSIM
           of Wang et al. 2004 with an 11x11 Gaussian window of standard
           deviation 1.5, C1 = 0.01^2, C2 = 0.03^2, zero outside the image)
  L_normal 1 - mean N . N_gt                                 (the normal loss
           equation of the appendix on normal back-propagation)
  L_depth  mean |D - D_gt|                                   (named in the
           total loss without a definition: read as an L1 term)
  L_seg    mean cross-entropy of softmax(O) against the label (section 3.3,
           semantic rendering); labels outside [0, C_o) add nothing
  L_K      mean |K - 1|                                      (the L_K equation;
           read as a mean, like the other terms)
  L_all    lambda_1 L_l1 + sum_x lambda_x |L_l1| / |L_x| L_x (the total-loss
           equation; the ratios are constants in the gradient, 0 when L_x = 0)
The gradient of the SSIM term is written out from the chain rule through the
windowed moments; the finite-difference pins in the tests check it.
"""
from __future__ import annotations

import numpy as np

C1 = 0.01 ** 2
C2 = 0.03 ** 2
RADIUS = 5
SIGMA = 1.5
DEFAULT_LAMBDAS = (1.0, 0.1, 0.1, 0.1, 0.1, 0.1)


def window():
    """Normalised 2-D Gaussian window, (2R+1) x (2R+1)."""
    d = np.arange(-RADIUS, RADIUS + 1, dtype=np.float64)
    g = np.exp(-d * d / (2.0 * SIGMA * SIGMA))
    g /= g.sum()
    return np.outer(g, g)


def window_sum(img, w=None):
    """out(p) = sum over offsets o of w(o) img(p + o), img zero outside: the 2-D
    windowed sum written directly over the window's offsets."""
    if w is None:
        w = window()
    H, W = img.shape
    pad = np.zeros((H + 2 * RADIUS, W + 2 * RADIUS))
    pad[RADIUS:RADIUS + H, RADIUS:RADIUS + W] = img
    out = np.zeros((H, W))
    for dy in range(2 * RADIUS + 1):
        for dx in range(2 * RADIUS + 1):
            out += w[dy, dx] * pad[dy:dy + H, dx:dx + W]
    return out


def ssim_parts(x, y):
    """SSIM map of one channel and the moments it is built from."""
    mx, my = window_sum(x), window_sum(y)
    exx, eyy, exy = window_sum(x * x), window_sum(y * y), window_sum(x * y)
    sxx, syy, sxy = exx - mx * mx, eyy - my * my, exy - mx * my
    A1, A2 = 2 * mx * my + C1, 2 * sxy + C2
    B1, B2 = mx * mx + my * my + C1, sxx + syy + C2
    return A1 * A2 / (B1 * B2), dict(mx=mx, my=my, A1=A1, A2=A2, B1=B1, B2=B2)


def ssim_map(x, y):
    return ssim_parts(np.asarray(x, np.float64), np.asarray(y, np.float64))[0]


def ssim_grad(x, y, gS):
    """d(sum_p gS(p) SSIM(p)) / dx for one channel.  The SSIM at p depends on
    x through mu_x(p) = sum G x, E[x^2](p) = sum G x^2 and E[xy](p) = sum G x y;
    its partials with respect to those three moments are back-projected with the
    (symmetric) window."""
    S, m = ssim_parts(x, y)
    iB = 1.0 / (m["B1"] * m["B2"])
    dA1, dA2 = m["A2"] * iB, m["A1"] * iB
    dB1, dB2 = -S / m["B1"], -S / m["B2"]
    mx, my = m["mx"], m["my"]
    # A1 = 2 mx my + C1, A2 = 2 (Exy - mx my) + C2,
    # B1 = mx^2 + my^2 + C1, B2 = (Exx - mx^2) + (Eyy - my^2) + C2
    d_mu = gS * (2 * my * dA1 - 2 * my * dA2 + 2 * mx * dB1 - 2 * mx * dB2)
    d_exx = gS * dB2
    d_exy = gS * 2 * dA2
    return window_sum(d_mu) + 2 * x * window_sum(d_exx) + y * window_sum(d_exy)


def cross_entropy(logits, label):
    """Per-pixel cross-entropy and its gradient for [C][H][W] logits."""
    z = np.asarray(logits, np.float64)
    C = z.shape[0]
    zmax = z.max(axis=0)
    e = np.exp(z - zmax)
    se = e.sum(axis=0)
    lab = np.asarray(label, np.int64)
    ok = (lab >= 0) & (lab < C)
    safe = np.where(ok, lab, 0)
    picked = np.take_along_axis(z, safe[None], axis=0)[0]
    ce = np.where(ok, zmax + np.log(se) - picked, 0.0)
    onehot = (np.arange(C)[:, None, None] == safe[None]).astype(np.float64)
    grad = np.where(ok[None], e / se - onehot, 0.0)
    return ce, grad


def total_loss(outs, gts, lambdas=DEFAULT_LAMBDAS, balance=True):
    """outs/gts: per-view dicts (gt keys rgb and optional depth, normal,
    label).  Returns (dict of the 8 values, per-view gradient dicts with keys
    rgb, depth, kmap, normal, sem)."""
    P = sum(int(np.asarray(o["kmap"]).size) for o in outs)
    has = dict(normal=gts[0].get("normal") is not None, depth=gts[0].get("depth") is not None,
               seg=gts[0].get("label") is not None)
    s = dict(l1=0.0, ssim=0.0, normal=0.0, depth=0.0, seg=0.0, K=0.0)
    for o, t in zip(outs, gts):
        c, cg = np.asarray(o["rgb"], np.float64), np.asarray(t["rgb"], np.float64)
        s["l1"] += np.abs(c - cg).sum()
        s["ssim"] += sum(ssim_map(c[k], cg[k]).sum() for k in range(3))
        if has["normal"]:
            s["normal"] += (np.asarray(o["normal"], np.float64) * np.asarray(t["normal"], np.float64)).sum()
        if has["depth"]:
            s["depth"] += np.abs(np.asarray(o["depth"], np.float64) - np.asarray(t["depth"], np.float64)).sum()
        if has["seg"]:
            s["seg"] += cross_entropy(o["sem"], t["label"])[0].sum()
        s["K"] += np.abs(np.asarray(o["kmap"], np.float64) - 1.0).sum()
    L = dict(l1=s["l1"] / (3 * P), ssim=1.0 - s["ssim"] / (3 * P),
             normal=(1.0 - s["normal"] / P) if has["normal"] else 0.0,
             depth=s["depth"] / P if has["depth"] else 0.0, seg=s["seg"] / P if has["seg"] else 0.0, K=s["K"] / P)
    names = ("l1", "ssim", "normal", "depth", "seg", "K")
    on = dict(l1=True, ssim=True, normal=has["normal"], depth=has["depth"], seg=has["seg"], K=True)
    w = {}
    for n in names:
        if n == "l1" or not balance:
            w[n] = 1.0
        else:
            w[n] = abs(L["l1"]) / abs(L[n]) if L[n] != 0 else 0.0
        if not on[n]:
            w[n] = 0.0
    L["all"] = sum(lambdas[k] * w[n] * L[n] for k, n in enumerate(names))
    L["ssim_mean"] = s["ssim"] / (3 * P)
    lam = dict(zip(names, lambdas))
    grads = []
    for o, t in zip(outs, gts):
        c, cg = np.asarray(o["rgb"], np.float64), np.asarray(t["rgb"], np.float64)
        H, W = c.shape[1:]
        g = {}
        g_ssim = np.stack([ssim_grad(c[k], cg[k], np.ones((H, W))) for k in range(3)])
        g["rgb"] = lam["l1"] * w["l1"] * np.sign(c - cg) / (3 * P) - lam["ssim"] * w["ssim"] * g_ssim / (3 * P)
        g["kmap"] = lam["K"] * w["K"] * np.sign(np.asarray(o["kmap"], np.float64) - 1.0) / P
        g["depth"] = (lam["depth"] * w["depth"] * np.sign(np.asarray(o["depth"], np.float64) -
                                                          np.asarray(t["depth"], np.float64)) / P
                      if has["depth"] else np.zeros((H, W)))
        g["normal"] = (-lam["normal"] * w["normal"] * np.asarray(t["normal"], np.float64) / P
                       if has["normal"] else np.zeros((3, H, W)))
        sem = np.asarray(o["sem"], np.float64)
        g["sem"] = (lam["seg"] * w["seg"] * cross_entropy(sem, t["label"])[1] / P
                    if has["seg"] else np.zeros_like(sem))
        grads.append(g)
    return L, grads
