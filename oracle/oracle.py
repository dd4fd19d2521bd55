"""Python front end of the FP64 CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the
benchmark's CPU-baseline leg, never by the product package.  It shares no code
with the HIP path.  Inputs are the float32 arrays of the seeded scene generator,
promoted to float64 here; every arithmetic step of the method runs in oracle.c
(in double precision) except the tile binning reference below, which is the
plain definition written with numpy.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

OPTS_DEFAULT = dict(step1=1, step2=2, lambda_=0.5, orient_sign=1, prune_Tk=0.0, eps_n=1e-9, depth_mode=0)

NS_BORDER, NS_ZERO, NS_VALID = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (-O2, no fast-math, OpenMP) into liboracle.so."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-fPIC",
                           "-shared", "-std=c11", "-Wall", "-o", tmp, SRC, "-lm"])
    os.replace(tmp, LIB)
    return LIB


class _Cam(C.Structure):
    _fields_ = [("W", C.c_int), ("H", C.c_int), ("fx", C.c_double), ("fy", C.c_double),
                ("cx", C.c_double), ("cy", C.c_double), ("R", C.c_double * 9), ("t", C.c_double * 3),
                ("z_near", C.c_double)]


class _Gs(C.Structure):
    _fields_ = [("N", C.c_int64), ("sh_deg", C.c_int), ("C_o", C.c_int),
                ("mean", C.c_void_p), ("quat", C.c_void_p), ("log_scale", C.c_void_p),
                ("opacity_logit", C.c_void_p), ("mask_logit", C.c_void_p), ("sh", C.c_void_p),
                ("sem", C.c_void_p)]


class _Opt(C.Structure):
    _fields_ = [("step1", C.c_int), ("step2", C.c_int), ("lambda_", C.c_double),
                ("orient_sign", C.c_int), ("prune_Tk", C.c_double), ("eps_n", C.c_double),
                ("depth_mode", C.c_int)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        _lib = C.CDLL(LIB)
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


class _Scene:
    """Holds float64 copies of the Gaussian arrays and the ctypes struct."""

    def __init__(self, g):
        self.arrs = {k: np.ascontiguousarray(g[k], dtype=np.float64)
                     for k in ("mean", "quat", "log_scale", "opacity_logit", "mask_logit", "sh", "sem")}
        self.N, self.sh_deg, self.C_o = int(g["N"]), int(g["sh_deg"]), int(g["C_o"])
        a = self.arrs
        self.s = _Gs(self.N, self.sh_deg, self.C_o, _p(a["mean"]), _p(a["quat"]), _p(a["log_scale"]),
                     _p(a["opacity_logit"]), _p(a["mask_logit"]), _p(a["sh"]), _p(a["sem"]))


def _cam(cam):
    c = _Cam()
    c.W, c.H = int(cam["W"]), int(cam["H"])
    c.fx, c.fy, c.cx, c.cy = (float(cam[k]) for k in ("fx", "fy", "cx", "cy"))
    R = np.asarray(cam["R"], dtype=np.float64).reshape(9)
    t = np.asarray(cam["t"], dtype=np.float64).reshape(3)
    for i in range(9):
        c.R[i] = float(R[i])
    for i in range(3):
        c.t[i] = float(t[i])
    c.z_near = float(cam.get("z_near", 0.2))
    return c


def _opt(opts=None):
    o = dict(OPTS_DEFAULT)
    if opts:
        for k, v in opts.items():
            o["lambda_" if k == "lambda" else k] = v
    return _Opt(int(o["step1"]), int(o["step2"]), float(o["lambda_"]), int(o["orient_sign"]),
                float(o["prune_Tk"]), float(o["eps_n"]), int(o["depth_mode"]))


def _scene(g):
    return g if isinstance(g, _Scene) else _Scene(g)


def project(g, cam, opts=None):
    """Per-Gaussian projection of one view (EWA footprint, colour, depth key)."""
    S = _scene(g)
    N = S.N
    out = dict(visible=np.zeros(N, np.int32), ambiguous=np.zeros(N, np.int32),
               mean2d=np.zeros((N, 2)), conic=np.zeros((N, 3)), cov2d=np.zeros((N, 3)),
               opacity=np.zeros(N), k=np.zeros(N), rgb=np.zeros((N, 3)), rgb_raw=np.zeros((N, 3)),
               depth=np.zeros(N), radius=np.zeros((N, 2)))
    L = lib()
    L.orc_project(C.byref(S.s), C.byref(_cam(cam)), C.byref(_opt(opts)),
                  *[_p(out[k]) for k in ("visible", "ambiguous", "mean2d", "conic", "cov2d", "opacity", "k",
                                         "rgb", "rgb_raw", "depth", "radius")])
    return out


def render(g, cam, opts=None, path=1, pixmask=None):
    """Forward maps of one view: rgb [3][H][W], depth, kmap, sem [C_o][H][W],
    T_final, last_id (id of the last contributor, -1 if none), n_frag,
    n_clamped, term_id (id of the fragment at which the walk stops because it
    would take T below 1e-4, -1 if the walk reaches the end of the list) and
    the per-pixel decision margins."""
    S = _scene(g)
    H, W = int(cam["H"]), int(cam["W"])
    out = dict(rgb=np.zeros((3, H, W)), depth=np.zeros((H, W)), kmap=np.zeros((H, W)),
               sem=np.zeros((S.C_o, H, W)), T_final=np.ones((H, W)), last_id=np.full((H, W), -1, np.int32),
               n_frag=np.zeros((H, W), np.int32), n_clamped=np.zeros((H, W), np.int32),
               margin=np.full((H, W), np.inf), grad_margin=np.full((H, W), np.inf),
               term_id=np.full((H, W), -1, np.int32))
    pm = None if pixmask is None else np.ascontiguousarray(pixmask, dtype=np.uint8)
    rc = lib().orc_render(C.byref(S.s), C.byref(_cam(cam)), C.byref(_opt(opts)), int(path), _p(pm),
                          *[_p(out[k]) for k in ("rgb", "depth", "kmap", "sem", "T_final", "last_id",
                                                 "n_frag", "n_clamped", "margin", "grad_margin", "term_id")])
    if rc != 0:
        raise RuntimeError(f"orc_render failed ({rc})")
    return out


def normals(depth, cam, opts=None, pixmask=None):
    """Alg. normal_estimation on a depth image: normal [3][H][W] (world frame),
    state per pixel (low 2 bits: 0 border, 1 degenerate, 2 valid; bit 2: the
    view-facing flip was applied; bit 3: n2 was sign-flipped for consistency)
    and decision margins."""
    H, W = int(cam["H"]), int(cam["W"])
    d = np.ascontiguousarray(depth, dtype=np.float64).reshape(H, W)
    out = dict(normal=np.zeros((3, H, W)), state=np.zeros((H, W), np.int32), margin=np.full((H, W), np.inf))
    pm = None if pixmask is None else np.ascontiguousarray(pixmask, dtype=np.uint8)
    lib().orc_normals(_p(d), C.byref(_cam(cam)), C.byref(_opt(opts)), _p(pm),
                      _p(out["normal"]), _p(out["state"]), _p(out["margin"]))
    return out


def normal_backward(depth, cam, dnormal, opts=None):
    """Alg. normal_gradient: dL/dN [3][H][W] -> dL/dD [H][W] at the given depth."""
    H, W = int(cam["H"]), int(cam["W"])
    d = np.ascontiguousarray(depth, dtype=np.float64).reshape(H, W)
    dn = np.ascontiguousarray(dnormal, dtype=np.float64).reshape(3, H, W)
    gD = np.zeros((H, W))
    lib().orc_normal_backward(_p(d), C.byref(_cam(cam)), C.byref(_opt(opts)), _p(dn), _p(gD))
    return gD


def zero_grads(g):
    if isinstance(g, _Scene):
        N, C_o, nc = g.N, g.C_o, (g.sh_deg + 1) ** 2
    else:
        N, C_o = int(g["N"]), int(g["C_o"])
        nc = (int(g["sh_deg"]) + 1) ** 2
    return dict(mean=np.zeros((3, N)), quat=np.zeros((4, N)), log_scale=np.zeros((3, N)),
                opacity_logit=np.zeros(N), mask_logit=np.zeros(N), sh=np.zeros((nc, 3, N)),
                sem=np.zeros((N, C_o)))


def backward(g, cam, up, depth, opts=None, path=1, pixmask=None, grads=None):
    """Gradients of L = <up, outputs> for one view, ADDED to `grads` (created if
    None).  `up` holds planar upstream maps rgb/depth/kmap/normal/sem; `depth` is
    the forward depth image.  Returns (grads, gD) where gD = dL/dD + normal branch."""
    S = _scene(g)
    H, W = int(cam["H"]), int(cam["W"])
    gr = zero_grads(g) if grads is None else grads
    f64 = lambda a: np.ascontiguousarray(a, dtype=np.float64)
    d = f64(depth).reshape(H, W)
    ups = dict(rgb=f64(up["rgb"]).reshape(3, H, W), depth=f64(up["depth"]).reshape(H, W),
               kmap=f64(up["kmap"]).reshape(H, W), normal=f64(up["normal"]).reshape(3, H, W),
               sem=f64(up["sem"]).reshape(S.C_o, H, W))
    gD = np.zeros((H, W))
    pm = None if pixmask is None else np.ascontiguousarray(pixmask, dtype=np.uint8)
    rc = lib().orc_backward(C.byref(S.s), C.byref(_cam(cam)), C.byref(_opt(opts)), int(path), _p(pm), _p(d),
                            _p(ups["rgb"]), _p(ups["depth"]), _p(ups["kmap"]), _p(ups["normal"]), _p(ups["sem"]),
                            *[_p(gr[k]) for k in ("mean", "quat", "log_scale", "opacity_logit", "mask_logit",
                                                  "sh", "sem")], _p(gD))
    if rc != 0:
        raise RuntimeError(f"orc_backward failed ({rc})")
    return gr, gD


def forward_all(g, cams, opts=None, path=1):
    """Every output of every view: render + normals."""
    S = _scene(g)
    outs = []
    for cam in cams:
        o = render(S, cam, opts, path)
        n = normals(o["depth"], cam, opts)
        o["normal"], o["nstate"], o["nmargin"] = n["normal"], n["state"], n["margin"]
        outs.append(o)
    return outs


def backward_all(g, cams, ups, outs, opts=None, path=1):
    """Parameter gradients of L = sum over views of <up_v, outputs_v>."""
    S = _scene(g)
    gr = zero_grads(g)
    gDs = []
    for cam, up, o in zip(cams, ups, outs):
        _, gD = backward(S, cam, up, o["depth"], opts, path, grads=gr)
        gDs.append(gD)
    return gr, gDs


def loss(g, cams, ups, opts=None, path=1):
    """L = sum_v <up_v, (rgb, depth, kmap, normal, sem)_v> in float64."""
    outs = forward_all(g, cams, opts, path)
    L = 0.0
    for up, o in zip(ups, outs):
        for k in ("rgb", "depth", "kmap", "normal", "sem"):
            L += float(np.sum(np.asarray(up[k], np.float64).reshape(o[k].shape) * o[k]))
    return L, outs


def sh_basis(deg, d):
    Y = np.zeros(16)
    dY = np.zeros(48)
    dd = np.ascontiguousarray(d, dtype=np.float64)
    lib().orc_sh_basis(int(deg), _p(dd), _p(Y), _p(dY))
    return Y, dY.reshape(16, 3)


def fragment_depth(g, cam, i, u, v, opts=None):
    """Literal ray-ellipsoid midpoint depth of Gaussian i at (u, v): returns
    (d, t_mid, a, b, c) of the unit-sphere quadratic."""
    S = _scene(g)
    out = np.zeros(5)
    lib().orc_fragment_depth(C.byref(S.s), C.byref(_cam(cam)), C.byref(_opt(opts)), C.c_int64(int(i)),
                             C.c_double(float(u)), C.c_double(float(v)), _p(out))
    return out


def max_threads():
    return int(lib().orc_max_threads())


def set_threads(n):
    """OpenMP thread count of later oracle calls."""
    lib().orc_set_threads(int(n))


# ------------------------------------------------------------------ binning
ALPHA_MIN = 1.0 / 255.0


def tile_pairs(g, cam, opts, tile, tile_base=0, delta=1e-5):
    """Plain definition of the (tile, Gaussian) pairs of one view: a Gaussian
    belongs to a tile's list when at least one pixel (u, v) of that tile has
    alpha = min(0.99, o exp(-q/2)) >= 1/255 (section 3.4: the per-tile lists of
    the tile-based rasterizer hold the Gaussians that can reach the tile's
    pixels), with the FP64 footprint (2D mean, conic, opacity) of project().
    Pixels whose alpha lies within delta (relative) of 1/255, and Gaussians with
    an ambiguous cull, only make a pair optional.  Every pixel of the opacity-
    aware box (A11) plus two pixels is tested, which holds the whole
    alpha >= 1/255 ellipse.

    Returns dict(required, optional: int64 codes tile * N + id (global tile
    ids, tile_base added), key: float32 camera depth per Gaussian (the blend-
    order key), visible: bool per Gaussian)."""
    N = int(g["N"]) if not isinstance(g, _Scene) else g.N
    P = project(g, cam, opts)
    W, H = int(cam["W"]), int(cam["H"])
    tw, th = tile
    tiles_x = (W + tw - 1) // tw
    vis = P["visible"].astype(bool) & (P["depth"] > 0)
    amb = P["ambiguous"].astype(bool)
    idx = np.nonzero(vis | amb & (P["depth"] > 0))[0]
    mx, my = P["mean2d"][idx, 0], P["mean2d"][idx, 1]
    rx, ry = P["radius"][idx, 0] + 2.0, P["radius"][idx, 1] + 2.0
    x0 = np.clip(np.floor(mx - rx), 0, W - 1).astype(np.int64)
    x1 = np.clip(np.ceil(mx + rx), 0, W - 1).astype(np.int64)
    y0 = np.clip(np.floor(my - ry), 0, H - 1).astype(np.int64)
    y1 = np.clip(np.ceil(my + ry), 0, H - 1).astype(np.int64)
    inside = (mx + rx >= 0) & (mx - rx <= W - 1) & (my + ry >= 0) & (my - ry <= H - 1)
    w = np.where(inside, x1 - x0 + 1, 0)
    h = np.where(inside, y1 - y0 + 1, 0)
    cnt = w * h
    req, opt_ = [], []
    # chunks of Gaussians keep the pixel arrays small
    bounds = np.searchsorted(np.cumsum(cnt), np.arange(0, int(cnt.sum()) + 4_000_000, 4_000_000))
    for a, b in zip(bounds[:-1], bounds[1:]):
        if b <= a:
            continue
        sl = slice(a, b)
        c = cnt[sl]
        k = np.repeat(np.arange(a, b), c)
        pos = np.arange(int(c.sum())) - np.repeat(np.cumsum(c) - c, c)
        u = x0[k] + pos % np.maximum(w[k], 1)
        v = y0[k] + pos // np.maximum(w[k], 1)
        gi = idx[k]
        dx, dy = u - P["mean2d"][gi, 0], v - P["mean2d"][gi, 1]
        ca, cb, cc = P["conic"][gi, 0], P["conic"][gi, 1], P["conic"][gi, 2]
        q = ca * dx * dx + 2.0 * cb * dx * dy + cc * dy * dy
        alpha = np.minimum(0.99, P["opacity"][gi] * np.exp(-0.5 * q))
        near = np.abs(alpha - ALPHA_MIN) <= delta * ALPHA_MIN
        code = (tile_base + (v // th) * tiles_x + (u // tw)) * N + gi
        hit = alpha >= ALPHA_MIN
        sure = hit & ~near & vis[gi] & ~amb[gi]
        req.append(np.unique(code[sure]))
        opt_.append(np.unique(code[(hit | near) & ~sure]))
    cat = lambda xs: np.unique(np.concatenate(xs)) if xs else np.zeros(0, np.int64)
    required = cat(req)
    optional = np.setdiff1d(cat(opt_), required)
    return dict(required=required, optional=optional, key=P["depth"].astype(np.float32), visible=vis)


# ------------------------------------------------------------------ pruning
def prune(g, T_k, reset=True, states=()):
    """Differentiable pruning (section 3.3, "Pruning"): keep the Gaussians with
    |k - 1| <= T_k, k = sigmoid(mask_logit) (FP64, T_k rounded to FP32 as the
    option is), compacted in index order; with reset, the kept mask logits
    become float32(ln 9), i.e. k = 0.9.  `states` are dicts of arrays laid out
    like the parameters.  Returns (pruned dict, pruned states, keep mask,
    ambiguity mask: decisions within 1e-12 relative of the threshold)."""
    N = int(g["N"])
    m = np.asarray(g["mask_logit"], np.float64).reshape(N)
    dev = np.abs(1.0 / (1.0 + np.exp(-m)) - 1.0)
    T = float(np.float32(T_k))
    keep = dev <= T
    amb = np.abs(dev - T) <= 1e-12 * max(T, 1e-300)

    def compact(d):
        out = {}
        for k in ("mean", "quat", "log_scale", "opacity_logit", "mask_logit", "sh", "sem"):
            a = d.get(k)
            if a is None:
                out[k] = None
                continue
            a = np.asarray(a)
            out[k] = np.ascontiguousarray(a[keep] if k == "sem" else a[..., keep])
        return out

    res = compact(g)
    res.update(N=int(keep.sum()), sh_deg=int(g["sh_deg"]), C_o=int(g["C_o"]))
    if reset:
        res["mask_logit"] = np.full(res["N"], np.float32(np.log(9.0)), np.float32)
    return res, [compact(st) for st in states], keep, amb
