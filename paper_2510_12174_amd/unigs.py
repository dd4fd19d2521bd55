"""Python binding of libunigs (the gfx950 multimodal Gaussian rasterizer).

Argument marshalling only: every step of the rendering path runs in the HIP
kernels behind the C ABI declared in include/unigs.h.  PyTorch provides device
memory and the stream.  The functions ugs_* mirror the C entry points one to
one; `Rasterizer` sequences them for the per-view and batched forms, and
`RasterizeFunction` is the torch.autograd.Function around forward/backward.

There is no fallback: if libunigs.so is missing or no GPU is present, loading
raises.
"""
from __future__ import annotations

import ctypes as C
import json
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(PKG, "libunigs.so")

UGS_OK = 0
UGS_ERR_INVALID_ARG = -1
UGS_ERR_UNSUPPORTED = -2
UGS_ERR_CAPACITY = -3
UGS_ERR_HIP = -4
UGS_ERR_NOT_CAPTURED = -5
UGS_ERR_STATE = -6
UGS_MAX_CHANNELS = 256
UGS_MAX_VIEWS = 64

EXPORTS = ["ugs_default_options", "ugs_create", "ugs_destroy", "ugs_set_options", "ugs_workspace_size",
           "ugs_project", "ugs_bin_sort", "ugs_check_overflow", "ugs_render_fwd", "ugs_render_bwd",
           "ugs_step_capture", "ugs_step_replay", "ugs_autotune", "ugs_pair_count", "ugs_status_string",
           "ugs_last_hip_error", "ugs_enable_counters", "ugs_read_counters", "ugs_debug_buffer", "ugs_time_stage",
           "ugs_prune_scratch_size", "ugs_prune", "ugs_prune_noalloc", "ugs_default_loss_options",
           "ugs_loss_scratch_size", "ugs_loss"]


class UgsError(RuntimeError):
    def __init__(self, code, what, detail=""):
        self.code = code
        super().__init__(f"{what} failed: {code} ({status_string(code)}) {detail}".strip())


class ugs_camera(C.Structure):
    _fields_ = [("W", C.c_int), ("H", C.c_int), ("fx", C.c_float), ("fy", C.c_float), ("cx", C.c_float),
                ("cy", C.c_float), ("R", C.c_float * 9), ("t", C.c_float * 3), ("z_near", C.c_float)]


class ugs_gaussians(C.Structure):
    _fields_ = [("N", C.c_int64), ("sh_deg", C.c_int), ("C_o", C.c_int)] + \
               [(k, C.c_void_p) for k in ("mean", "quat", "log_scale", "opacity_logit", "mask_logit", "sh", "sem")]


class ugs_gaussian_grads(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("mean", "quat", "log_scale", "opacity_logit", "mask_logit", "sh", "sem")]


class ugs_outputs(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("rgb", "depth", "kmap", "normal", "sem", "T_final", "n_contrib")]


class ugs_upstream(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("rgb", "depth", "kmap", "normal", "sem", "normal_target", "normal_scale",
                                          "sem_label", "sem_scale")]


class ugs_options(C.Structure):
    _fields_ = [("tile_w", C.c_int), ("tile_h", C.c_int), ("batch", C.c_int), ("step1", C.c_int),
                ("step2", C.c_int), ("lambda_", C.c_float), ("orient_sign", C.c_int), ("prune_Tk", C.c_float),
                ("depth_mode", C.c_int), ("half_outputs", C.c_int), ("sem_bf16x3", C.c_int)]


class ugs_targets(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("rgb", "depth", "normal", "label")]


class ugs_loss_options(C.Structure):
    _fields_ = [("lambda_", C.c_float * 6), ("balance", C.c_int)]


LOSS_NAMES = ("l1", "ssim", "normal", "depth", "seg", "K", "all", "ssim_mean",
              "coef_l1", "coef_ssim", "coef_normal", "coef_depth", "coef_seg", "coef_K")
UGS_LOSS_VALUES = 14

_lib = None


def lib():
    """Loads libunigs.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise ImportError(f"{LIB} not found: build it with paper_2510_12174_amd/build.py "
                              "(or __graft_entry__.build())")
        L = C.CDLL(LIB)
        P = C.c_void_p
        L.ugs_default_options.argtypes = [C.POINTER(ugs_options)]
        L.ugs_default_options.restype = None
        L.ugs_create.argtypes = [C.POINTER(P), C.POINTER(ugs_options)]
        L.ugs_destroy.argtypes = [P]
        L.ugs_destroy.restype = None
        L.ugs_set_options.argtypes = [P, C.POINTER(ugs_options)]
        L.ugs_workspace_size.argtypes = [P, C.c_int64, C.c_int, C.c_int, C.POINTER(ugs_camera), C.c_int,
                                         C.c_int64, C.POINTER(C.c_size_t)]
        L.ugs_project.argtypes = [P, C.POINTER(ugs_gaussians), C.POINTER(ugs_camera), C.c_int, P, C.c_size_t, P]
        L.ugs_bin_sort.argtypes = [P, P, P, C.POINTER(C.c_int64)]
        L.ugs_check_overflow.argtypes = [P, P, P, C.POINTER(C.c_int64)]
        L.ugs_pair_count.argtypes = [P, P, P, C.POINTER(C.c_int64)]
        L.ugs_render_fwd.argtypes = [P, C.POINTER(ugs_gaussians), P, C.POINTER(ugs_outputs), P]
        L.ugs_render_bwd.argtypes = [P, C.POINTER(ugs_gaussians), P, C.POINTER(ugs_outputs),
                                     C.POINTER(ugs_upstream), C.POINTER(ugs_gaussian_grads), P]
        L.ugs_step_capture.argtypes = [P, C.POINTER(ugs_gaussians), C.POINTER(ugs_camera), C.c_int, P, C.c_size_t,
                                       C.POINTER(ugs_outputs), C.POINTER(ugs_upstream),
                                       C.POINTER(ugs_gaussian_grads), P]
        L.ugs_step_replay.argtypes = [P, P]
        L.ugs_autotune.argtypes = [P, C.POINTER(ugs_gaussians), C.POINTER(ugs_camera), C.c_int, P, C.c_size_t,
                                   C.POINTER(ugs_outputs), C.POINTER(ugs_upstream), C.POINTER(ugs_gaussian_grads), P,
                                   C.POINTER(ugs_options), C.POINTER(C.c_float)]
        L.ugs_status_string.argtypes = [C.c_int]
        L.ugs_status_string.restype = C.c_char_p
        L.ugs_last_hip_error.argtypes = [P]
        L.ugs_last_hip_error.restype = C.c_char_p
        L.ugs_enable_counters.argtypes = [P, C.c_int]
        L.ugs_read_counters.argtypes = [P, P, P, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        L.ugs_debug_buffer.argtypes = [P, P, C.c_int, P, C.POINTER(C.c_void_p), C.POINTER(C.c_int64)]
        L.ugs_time_stage.argtypes = [P, C.c_int, P, P]
        L.ugs_prune_scratch_size.argtypes = [C.c_int64, C.POINTER(C.c_size_t)]
        L.ugs_prune.argtypes = [C.POINTER(ugs_gaussians), C.POINTER(ugs_gaussian_grads), C.c_int,
                                C.POINTER(ugs_gaussians), C.POINTER(ugs_gaussian_grads), C.c_float, C.c_int, P,
                                C.c_size_t, C.POINTER(C.c_int64), P]
        L.ugs_prune_noalloc.argtypes = [C.POINTER(ugs_gaussians), C.POINTER(ugs_gaussian_grads), C.c_int,
                                        C.POINTER(ugs_gaussians), C.POINTER(ugs_gaussian_grads), C.c_float, C.c_int,
                                        C.POINTER(C.c_int64), P]
        L.ugs_default_loss_options.argtypes = [C.POINTER(ugs_loss_options)]
        L.ugs_default_loss_options.restype = None
        L.ugs_loss_scratch_size.argtypes = [C.POINTER(ugs_camera), C.c_int, C.POINTER(C.c_size_t)]
        L.ugs_loss.argtypes = [C.POINTER(ugs_camera), C.c_int, C.c_int, C.POINTER(ugs_outputs),
                               C.POINTER(ugs_targets), C.POINTER(ugs_loss_options), C.POINTER(ugs_upstream), P, P,
                               C.c_size_t, P]
        _lib = L
    return _lib


def status_string(code):
    try:
        return lib().ugs_status_string(int(code)).decode()
    except Exception:
        return "?"


# ---------------------------------------------------------------- marshalling
def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def make_cameras(cams):
    arr = (ugs_camera * len(cams))()
    for i, c in enumerate(cams):
        arr[i].W, arr[i].H = int(c["W"]), int(c["H"])
        arr[i].fx, arr[i].fy, arr[i].cx, arr[i].cy = (float(c[k]) for k in ("fx", "fy", "cx", "cy"))
        R = np.asarray(c["R"], np.float32).reshape(9)
        t = np.asarray(c["t"], np.float32).reshape(3)
        for k in range(9):
            arr[i].R[k] = float(R[k])
        for k in range(3):
            arr[i].t[k] = float(t[k])
        arr[i].z_near = float(c.get("z_near", 0.2))
    return arr


PARAM_KEYS = ("mean", "quat", "log_scale", "opacity_logit", "mask_logit", "sh", "sem")


def make_gaussians(g):
    """g: dict with N, sh_deg, C_o and contiguous float32 device tensors."""
    s = ugs_gaussians()
    s.N, s.sh_deg, s.C_o = int(g["N"]), int(g["sh_deg"]), int(g["C_o"])
    for k in PARAM_KEYS:
        t = g[k]
        _check_tensor(t, k)
        setattr(s, k, t.data_ptr())
    return s


def make_grads(d):
    s = ugs_gaussian_grads()
    for k in PARAM_KEYS:
        _check_tensor(d[k], "d" + k)
        setattr(s, k, d[k].data_ptr())
    return s


def _check_tensor(t, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype not in (torch.float32, torch.int32) \
            or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float32 CUDA tensor")


def check_map(t, name, dtype, numel):
    """Raises ValueError unless `t` is a contiguous CUDA tensor of `dtype` (a
    torch dtype) with `numel` elements: the C ABI reads raw pointers, so a wrong
    element type (int64 class labels read as int32 pairs), a strided view or a
    short map would be read wrongly or out of bounds."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name} must be a torch tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() != int(numel):
        raise ValueError(f"{name} must have {int(numel)} elements, got {t.numel()}")


def check_outputs(o, P, C_o, half=False, state=True):
    """Validates output planes for P pixels (all views) and C_o channels."""
    import torch
    mt = torch.float16 if half else torch.float32
    for k, n, dt in (("rgb", 3 * P, mt), ("depth", P, torch.float32), ("kmap", P, mt), ("normal", 3 * P, mt)):
        check_map(o.get(k), k, dt, n)
    if C_o > 0:
        check_map(o.get("sem"), "sem", mt, C_o * P)
    if state or o.get("T_final") is not None:
        check_map(o.get("T_final"), "T_final", torch.float32, P)
    if state or o.get("n_contrib") is not None:
        check_map(o.get("n_contrib"), "n_contrib", torch.int32, P)


def check_upstream(u, P, C_o):
    """Validates the upstream gradient maps (absent maps may be None)."""
    import torch
    f, i = torch.float32, torch.int32
    for k, n, dt in (("rgb", 3 * P, f), ("depth", P, f), ("kmap", P, f), ("normal", 3 * P, f),
                     ("sem", C_o * P, f), ("normal_target", 3 * P, f), ("normal_scale", 1, f),
                     ("sem_label", P, i), ("sem_scale", 1, f)):
        t = u.get(k) if u else None
        if t is not None and not (k == "sem" and C_o == 0):
            check_map(t, k, dt, n)


def make_outputs(o):
    s = ugs_outputs()
    for k in ("rgb", "depth", "kmap", "normal", "sem", "T_final", "n_contrib"):
        setattr(s, k, o[k].data_ptr() if o.get(k) is not None and o[k].numel() > 0 else None)
    return s


def make_upstream(u):
    s = ugs_upstream()
    for k in ("rgb", "depth", "kmap", "normal", "sem", "normal_target", "normal_scale", "sem_label", "sem_scale"):
        t = u.get(k) if u else None
        setattr(s, k, t.data_ptr() if t is not None and t.numel() > 0 else None)
    return s


def default_options(**kw):
    o = ugs_options()
    lib().ugs_default_options(C.byref(o))
    for k, v in kw.items():
        setattr(o, "lambda_" if k == "lambda" else k, v)
    return o


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _chk(rc, what, ctx=None):
    if rc != UGS_OK:
        detail = ""
        if ctx is not None:
            detail = lib().ugs_last_hip_error(ctx).decode()
        raise UgsError(rc, what, detail)


# ---------------------------------------------------------------- high level
def to_device(g, device="cuda"):
    """Seeded-scene dict (numpy) -> dict of contiguous float32 device tensors."""
    import torch
    out = dict(N=int(g["N"]), sh_deg=int(g["sh_deg"]), C_o=int(g["C_o"]))
    for k in PARAM_KEYS:
        a = np.asarray(g[k], np.float32)
        if k == "sem" and a.size == 0:
            a = np.zeros((int(g["N"]), 0), np.float32)
        out[k] = torch.from_numpy(np.ascontiguousarray(a)).to(device)
    return out


def zeros_like_params(g):
    import torch
    return {k: torch.zeros_like(g[k]) for k in PARAM_KEYS}


UGS_PRUNE_NOALLOC_MAX_N = 1 << 22


def prune(g, T_k, reset_k=True, states=(), noalloc=False):
    """Differentiable pruning (ugs_prune): returns (pruned parameter dict,
    list of pruned state dicts, kept count).  `states` are dicts with the
    parameter keys (None for absent arrays), laid out like the parameters.
    noalloc=True calls ugs_prune_noalloc (the library's own scratch array,
    N <= UGS_PRUNE_NOALLOC_MAX_N) instead of allocating a scratch buffer."""
    import torch
    N = int(g["N"])
    out = {k: torch.empty_like(g[k]) for k in PARAM_KEYS}
    outs_state = [{k: (torch.empty_like(st[k]) if st.get(k) is not None else None) for k in PARAM_KEYS}
                  for st in states]
    if not noalloc:
        nb = C.c_size_t()
        _chk(lib().ugs_prune_scratch_size(N, C.byref(nb)), "ugs_prune_scratch_size")
        scratch = torch.empty(int(nb.value), dtype=torch.uint8, device=g["mean"].device)
    gs = make_gaussians(g)
    os_ = make_grads(out)
    n_state = len(states)
    sin = (ugs_gaussians * max(n_state, 1))()
    sout = (ugs_gaussian_grads * max(n_state, 1))()
    for k_, (st, so) in enumerate(zip(states, outs_state)):
        sin[k_].N, sin[k_].sh_deg, sin[k_].C_o = N, int(g["sh_deg"]), int(g["C_o"])
        for key in PARAM_KEYS:
            setattr(sin[k_], key, st[key].data_ptr() if st.get(key) is not None else None)
            setattr(sout[k_], key, so[key].data_ptr() if so.get(key) is not None else None)
    nk = C.c_int64()
    if noalloc:
        _chk(lib().ugs_prune_noalloc(C.byref(gs), C.byref(os_), n_state, sin, sout, float(T_k), int(bool(reset_k)),
                                     C.byref(nk), _stream()), "ugs_prune_noalloc")
    else:
        _chk(lib().ugs_prune(C.byref(gs), C.byref(os_), n_state, sin, sout, float(T_k), int(bool(reset_k)),
                             C.c_void_p(scratch.data_ptr()), int(nb.value), C.byref(nk), _stream()), "ugs_prune")
    n = int(nk.value)

    def view(key, t):
        if t is None:
            return None
        if key == "sem":  # [N][C_o], row-major per Gaussian
            return t[:n]
        shape = tuple(g[key].shape[:-1])  # structure of arrays: rows packed at stride n
        rows = int(np.prod(shape)) if shape else 1
        return t.view(-1)[:rows * n].view(*shape, n)

    res = dict(N=n, sh_deg=int(g["sh_deg"]), C_o=int(g["C_o"]))
    for key in PARAM_KEYS:
        res[key] = view(key, out[key])
    res_states = [{key: view(key, so[key]) for key in PARAM_KEYS} for so in outs_state]
    return res, res_states, n


def loss_options(lambdas=None, balance=True):
    o = ugs_loss_options()
    lib().ugs_default_loss_options(C.byref(o))
    if lambdas is not None:
        for k in range(6):
            o.lambda_[k] = float(lambdas[k])
    o.balance = int(bool(balance))
    return o


class Loss:
    """The section-3.4 loss (ugs_loss) for a fixed set of views: owns the
    scratch buffer, the 8-float loss vector and the gradient maps, which are
    the upstream of Rasterizer.backward."""

    def __init__(self, cams, C_o, lambdas=None, balance=True, device="cuda", fuse_normal=False, fuse_seg=False):
        import torch
        self.cams_c = make_cameras(cams)
        self.V, self.C_o = len(cams), int(C_o)
        nb = C.c_size_t()
        _chk(lib().ugs_loss_scratch_size(self.cams_c, self.V, C.byref(nb)), "ugs_loss_scratch_size")
        self.scratch = torch.empty(int(nb.value), dtype=torch.uint8, device=device)
        self.nb = int(nb.value)
        self.losses = torch.zeros(UGS_LOSS_VALUES, dtype=torch.float32, device=device)
        P = pixel_offsets(cams)[-1]
        f = lambda n: torch.empty(n, dtype=torch.float32, device=device)
        # fuse_normal: no normal gradient map; the backward forms the cosine seed
        # itself from the target normals and the coefficient in losses[10]
        # fuse_seg: no semantic gradient map; the backward forms the
        # cross-entropy seed from the rendered logits, the labels and losses[12]
        self.fuse_normal, self.fuse_seg = bool(fuse_normal), bool(fuse_seg)
        self.grad = dict(rgb=f(3 * P), depth=f(P), kmap=f(P), normal=None if fuse_normal else f(3 * P),
                         sem=None if fuse_seg else f(max(self.C_o, 0) * P))
        self.opts = loss_options(lambdas, balance)

    def __call__(self, out, gt):
        """out: rasterizer outputs; gt: dict with rgb and optional depth,
        normal, label (int32).  Returns (losses tensor[8], gradient dict)."""
        import torch
        P = pixel_offsets_from(self.cams_c)
        check_outputs(out, P, self.C_o, state=False)
        for k, n, dt in (("rgb", 3 * P, torch.float32), ("depth", P, torch.float32),
                         ("normal", 3 * P, torch.float32), ("label", P, torch.int32)):
            if gt.get(k) is not None or k == "rgb":
                check_map(gt.get(k), "gt " + k, dt, n)
        t = ugs_targets()
        for k in ("rgb", "depth", "normal", "label"):
            v = gt.get(k)
            setattr(t, k, v.data_ptr() if v is not None else None)
        o, u = make_outputs(out), make_upstream(self.grad)
        _chk(lib().ugs_loss(self.cams_c, self.V, self.C_o, C.byref(o), C.byref(t), C.byref(self.opts), C.byref(u),
                            _ptr(self.losses), _ptr(self.scratch), self.nb, _stream()), "ugs_loss")
        if self.fuse_normal or self.fuse_seg:
            up = dict(self.grad)
            if self.fuse_normal and gt.get("normal") is not None:
                up.update(normal_target=gt["normal"], normal_scale=self.losses[10:11])
            if self.fuse_seg and gt.get("label") is not None:
                up.update(sem_label=gt["label"], sem_scale=self.losses[12:13])
            return self.losses, up
        return self.losses, self.grad


def pixel_offsets_from(cams_c):
    """Total pixel count of a ctypes camera array."""
    return sum(int(c.W) * int(c.H) for c in cams_c)


def pixel_offsets(cams):
    off = [0]
    for c in cams:
        off.append(off[-1] + int(c["W"]) * int(c["H"]))
    return off


def alloc_outputs(cams, C_o, device="cuda", state=True, half=False):
    """Output planes for all views; state=False leaves out T_final and
    n_contrib (forward-only use: the backward needs them); half=True makes the
    rgb, kmap, normal and sem planes float16 (for a rasterizer created with
    half_outputs=1)."""
    import torch
    P = pixel_offsets(cams)[-1]
    f = lambda n: torch.empty(n, dtype=torch.float32, device=device)
    h = (lambda n: torch.empty(n, dtype=torch.float16, device=device)) if half else f
    o = dict(rgb=h(3 * P), depth=f(P), kmap=h(P), normal=h(3 * P), sem=h(max(C_o, 0) * P))
    if state:
        o.update(T_final=f(P), n_contrib=torch.empty(P, dtype=torch.int32, device=device))
    return o


def split_views(flat, cams, channels):
    """Flat stacked planes -> list of [channels][H][W] views per camera."""
    off = pixel_offsets(cams)
    res = []
    for v, c in enumerate(cams):
        H, W = int(c["H"]), int(c["W"])
        res.append(flat[channels * off[v]:channels * off[v + 1]].view(channels, H, W))
    return res


class Rasterizer:
    """Owns a libunigs context, its workspace and the output buffers."""

    def __init__(self, **options):
        import torch
        self.torch = torch
        self.opts = default_options(**options)
        ctx = C.c_void_p()
        _chk(lib().ugs_create(C.byref(ctx), C.byref(self.opts)), "ugs_create")
        self.ctx = ctx
        self.ws = None
        self.ws_bytes = 0
        self.pair_cap = 0
        self._keep = []
        # projection generation: bumped by every projection of this context, so
        # that a backward can tell whether the workspace still holds the
        # projection of the forward it belongs to; bwd_consumed is set once a
        # backward has used that projection's gradient records
        self.generation = 0
        self.bwd_consumed = False

    def __del__(self):
        try:
            if getattr(self, "ctx", None):
                lib().ugs_destroy(self.ctx)
                self.ctx = None
        except Exception:
            pass

    def set_options(self, **options):
        for k, v in options.items():
            setattr(self.opts, "lambda_" if k == "lambda" else k, v)
        _chk(lib().ugs_set_options(self.ctx, C.byref(self.opts)), "ugs_set_options", self.ctx)
        self.generation += 1  # the context forgets its projection
        self.bwd_consumed = True

    def workspace_size(self, g, cams, pair_cap):
        n = C.c_size_t()
        cs = make_cameras(cams)
        _chk(lib().ugs_workspace_size(self.ctx, int(g["N"]), int(g["C_o"]), int(g["sh_deg"]), cs, len(cams),
                                      int(pair_cap), C.byref(n)), "ugs_workspace_size")
        return n.value

    def ensure_workspace(self, g, cams, pair_cap):
        need = self.workspace_size(g, cams, pair_cap)
        if self.ws is None or self.ws_bytes < need:
            self.ws = None
            self.ws = self.torch.empty(need + 256, dtype=self.torch.uint8, device="cuda")
            self.ws_bytes = need
        self.pair_cap = pair_cap
        base = self.ws.data_ptr()
        self.ws_ptr = C.c_void_p((base + 255) & ~255)

    def project_and_sort(self, g, cams, pair_cap=None):
        """S1-S4 with the pair-count read-back; grows the workspace and repeats on
        overflow.  Returns the pair count P."""
        cs = make_cameras(cams)
        gs = make_gaussians(g)
        cap = pair_cap or max(self.pair_cap, 1 << 16, 4 * int(g["N"]) * len(cams))
        for _ in range(4):
            self.ensure_workspace(g, cams, cap)
            s = _stream()
            self.generation += 1
            self.bwd_consumed = False
            _chk(lib().ugs_project(self.ctx, C.byref(gs), cs, len(cams), self.ws_ptr, self.ws_bytes, s),
                 "ugs_project", self.ctx)
            P = C.c_int64()
            rc = lib().ugs_bin_sort(self.ctx, self.ws_ptr, s, C.byref(P))
            if rc == UGS_ERR_CAPACITY:
                cap = int(P.value * 1.25) + 1024
                continue
            _chk(rc, "ugs_bin_sort", self.ctx)
            return int(P.value)
        raise UgsError(UGS_ERR_CAPACITY, "project_and_sort")

    def forward(self, g, cams, out=None):
        if out is None:
            out = alloc_outputs(cams, int(g["C_o"]), half=bool(self.opts.half_outputs))
        check_outputs(out, pixel_offsets(cams)[-1], int(g["C_o"]), half=bool(self.opts.half_outputs),
                      state=False)
        self.project_and_sort(g, cams)
        _chk(lib().ugs_render_fwd(self.ctx, C.byref(make_gaussians(g)), self.ws_ptr, C.byref(make_outputs(out)),
                                  _stream()), "ugs_render_fwd", self.ctx)
        return out

    def backward(self, g, out, up, grads=None):
        if grads is None:
            grads = zeros_like_params(g)
        P = int(out["depth"].numel())
        check_outputs(out, P, int(g["C_o"]))
        check_upstream(up, P, int(g["C_o"]))
        _chk(lib().ugs_render_bwd(self.ctx, C.byref(make_gaussians(g)), self.ws_ptr, C.byref(make_outputs(out)),
                                  C.byref(make_upstream(up)), C.byref(make_grads(grads)), _stream()),
             "ugs_render_bwd", self.ctx)
        self.bwd_consumed = True
        return grads

    def pair_count(self):
        P = C.c_int64()
        _chk(lib().ugs_pair_count(self.ctx, self.ws_ptr, _stream(), C.byref(P)), "ugs_pair_count", self.ctx)
        return int(P.value)

    def enable_counters(self, on=True):
        _chk(lib().ugs_enable_counters(self.ctx, int(on)), "ugs_enable_counters")

    def read_counters(self):
        e, c = C.c_int64(), C.c_int64()
        _chk(lib().ugs_read_counters(self.ctx, self.ws_ptr, _stream(), C.byref(e), C.byref(c)),
             "ugs_read_counters", self.ctx)
        return int(e.value), int(c.value)

    STAGES = dict(project=1, bin_sort=2, render_fwd=3, normal_fwd=4, normal_bwd=5, render_bwd=6, project_bwd=7)

    def time_stage(self, stage, ev_start=None, ev_stop=None):
        """Records the hipEvent_t handles ev_start/ev_stop around one stage's
        kernels in every later call (and in a step captured afterwards)."""
        st = self.STAGES[stage] if isinstance(stage, str) else int(stage)
        _chk(lib().ugs_time_stage(self.ctx, st, C.c_void_p(ev_start), C.c_void_p(ev_stop)), "ugs_time_stage")

    DEBUG = {"records": (0, "float32", 16), "rects": (1, "int32", 2), "touched": (2, "int32", 1),
             "keys": (3, "int32", 1), "vals": (4, "int32", 1), "ranges": (5, "int32", 2),
             "grad_records": (6, "float32", 16), "depth_grad": (7, "float32", 1),
             "tile_clock_fwd": (8, "int64", 2), "tile_clock_bwd": (9, "int64", 2),
             "activity_mask": (10, "int32", 1)}

    def debug_buffer(self, name):
        """Device tensor view of an internal workspace array (see ugs_debug_buffer)."""
        which, dt, width = self.DEBUG[name]
        ptr, cnt = C.c_void_p(), C.c_int64()
        _chk(lib().ugs_debug_buffer(self.ctx, self.ws_ptr, which, _stream(), C.byref(ptr), C.byref(cnt)),
             "ugs_debug_buffer", self.ctx)
        dtype = getattr(self.torch, dt)
        esize = self.torch.empty(0, dtype=dtype).element_size()
        off = int(ptr.value or self.ws.data_ptr()) - self.ws.data_ptr()
        n = int(cnt.value) * width
        return self.ws[off:off + n * esize].view(dtype).view(-1, width) if width > 1 else \
            self.ws[off:off + n * esize].view(dtype)

    # batched step ------------------------------------------------------
    def capture_step(self, g, cams, out, up, grads, margin=1.25):
        """Sizes the workspace from an eager pass (pair count x margin) and
        captures the whole fwd+bwd step for all views into one HIP graph; with
        up and grads both None, the forward-only step."""
        P = self.project_and_sort(g, cams)
        self.ensure_workspace(g, cams, max(int(P * margin) + 4096, self.pair_cap))
        self._cap_args = (g, cams, out, up, grads)
        fwd_only = up is None and grads is None
        self._keep = [make_gaussians(g), make_cameras(cams), make_outputs(out),
                      None if fwd_only else make_upstream(up), None if fwd_only else make_grads(grads)]
        gs, cs, os_, us, ds = self._keep
        # capture needs a non-default stream; the graph is launched later on
        # whatever stream is current
        torch = self.torch
        cur = torch.cuda.current_stream()
        side = torch.cuda.Stream()
        side.wait_stream(cur)
        with torch.cuda.stream(side):
            rc = lib().ugs_step_capture(self.ctx, C.byref(gs), cs, len(cams), self.ws_ptr, self.ws_bytes,
                                        C.byref(os_), C.byref(us) if us is not None else None,
                                        C.byref(ds) if ds is not None else None, C.c_void_p(side.cuda_stream))
        cur.wait_stream(side)
        _chk(rc, "ugs_step_capture", self.ctx)

    def replay(self):
        _chk(lib().ugs_step_replay(self.ctx, _stream()), "ugs_step_replay", self.ctx)
        self.generation += 1  # the captured step projects again
        self.bwd_consumed = True

    def replay_checked(self, margin=1.5):
        """Replays the captured step, then synchronises and checks that its
        pair count fitted the workspace (ugs_check_overflow).  If it did not (the
        step's outputs and gradients are then zero), captures the step again
        with room for the required pairs x margin, on the same tensors, and
        replays it.  Returns True when it re-captured."""
        self.replay()
        P = C.c_int64()
        rc = lib().ugs_check_overflow(self.ctx, self.ws_ptr, _stream(), C.byref(P))
        if rc != UGS_ERR_CAPACITY:
            _chk(rc, "ugs_check_overflow", self.ctx)
            return False
        self.pair_cap = max(self.pair_cap, int(P.value * margin) + 4096)
        self.capture_step(*self._cap_args, margin=margin)
        self.replay()
        return True

    def autotune(self, g, cams, out, up, grads, cache=None):
        """ugs_autotune, with its choice cached in a JSON file keyed by
        tune_key() (GPU architecture, channels, SH degree, Gaussian-count and
        megapixel buckets).  cache: a path, False for no cache, or None for
        $UNIGS_TUNE_CACHE (default ~/.cache/unigs/autotune.json).  A cached
        choice is applied without timing (the result then has cached=True)."""
        path = tune_cache_path(cache)
        key = tune_key(g, cams)
        if path:
            hit = _read_json(path).get(key)
            if hit:
                self.set_options(tile_w=int(hit["tile_w"]), tile_h=int(hit["tile_h"]), batch=int(hit["batch"]))
                return dict(hit, cached=True)
        res = self._autotune(g, cams, out, up, grads)
        if path:
            d = _read_json(path)
            d[key] = res
            os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
            tmp = path + ".tmp"
            with open(tmp, "w") as f:
                json.dump(d, f, indent=1, sort_keys=True)
            os.replace(tmp, path)
        return dict(res, cached=False)

    def _autotune(self, g, cams, out, up, grads):
        P = self.project_and_sort(g, cams)
        # the smallest tile needs the most pairs: leave room for it (candidates
        # that still overflow are skipped by the library)
        self.ensure_workspace(g, cams, max(int(P * 4.0) + 4096, self.pair_cap))
        chosen = ugs_options()
        ms = C.c_float()
        rc = lib().ugs_autotune(self.ctx, C.byref(make_gaussians(g)), make_cameras(cams), len(cams), self.ws_ptr,
                                self.ws_bytes, C.byref(make_outputs(out)), C.byref(make_upstream(up)),
                                C.byref(make_grads(grads)), _stream(), C.byref(chosen), C.byref(ms))
        self.generation += 1  # the candidates' steps overwrote the workspace
        self.bwd_consumed = True
        _chk(rc, "ugs_autotune", self.ctx)
        self.opts = chosen
        return dict(tile_w=chosen.tile_w, tile_h=chosen.tile_h, batch=chosen.batch, ms=float(ms.value))


def tune_key(g, cams):
    """Autotune cache key: GPU architecture, C_o, SH degree, and power-of-two
    buckets of the Gaussian count and of the pixel count."""
    import torch
    arch = torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName.split(":")[0]
    n = max(int(g["N"]), 1)
    px = max(sum(int(c["W"]) * int(c["H"]) for c in cams), 1)
    return f"{arch}|C_o={int(g['C_o'])}|sh={int(g['sh_deg'])}|N~2^{n.bit_length()}|px~2^{px.bit_length()}"


def tune_cache_path(cache=None):
    if cache is False:
        return None
    if cache:
        return str(cache)
    return os.environ.get("UNIGS_TUNE_CACHE") or os.path.join(os.path.expanduser("~"), ".cache", "unigs",
                                                              "autotune.json")


def _read_json(path):
    try:
        with open(path) as f:
            d = json.load(f)
        return d if isinstance(d, dict) else {}
    except (OSError, ValueError):
        return {}


def _autograd_function():
    import torch

    class RasterizeFunction(torch.autograd.Function):
        """Differentiable multimodal render of all views.  Inputs are the seven
        parameter tensors; outputs are the stacked planes (rgb, depth, kmap,
        normal, sem).  The backward recomputes transmittance from the saved
        T_final (no per-fragment state is stored)."""

        @staticmethod
        def forward(ctx, rast, meta, cams, mean, quat, log_scale, opacity_logit, mask_logit, sh, sem):
            g = dict(meta, mean=mean.contiguous(), quat=quat.contiguous(), log_scale=log_scale.contiguous(),
                     opacity_logit=opacity_logit.contiguous(), mask_logit=mask_logit.contiguous(),
                     sh=sh.contiguous(), sem=sem.contiguous())
            out = rast.forward(g, cams)
            ctx.rast, ctx.g, ctx.out, ctx.cams = rast, g, out, cams
            ctx.generation = rast.generation
            ctx.mark_non_differentiable(out["T_final"], out["n_contrib"])
            return out["rgb"], out["depth"], out["kmap"], out["normal"], out["sem"], out["T_final"], out["n_contrib"]

        @staticmethod
        def backward(ctx, d_rgb, d_depth, d_kmap, d_normal, d_sem, _dT, _dn):
            up = {}
            for k, t in (("rgb", d_rgb), ("depth", d_depth), ("kmap", d_kmap), ("normal", d_normal),
                         ("sem", d_sem)):
                up[k] = None if t is None else t.contiguous()
            rast = ctx.rast
            if rast.generation != ctx.generation or rast.bwd_consumed:
                # the workspace no longer holds this forward's projection (another
                # render on the same rasterizer, or a second backward of this one):
                # project and sort again (deterministic: the same records and tile
                # lists the saved T_final and n_contrib index)
                rast.project_and_sort(ctx.g, ctx.cams)
            grads = rast.backward(ctx.g, ctx.out, up)
            return (None, None, None, grads["mean"], grads["quat"], grads["log_scale"], grads["opacity_logit"],
                    grads["mask_logit"], grads["sh"], grads["sem"])

    return RasterizeFunction


_RF = None


def rasterize(rast, g, cams):
    """Differentiable render: returns dict of stacked output planes."""
    global _RF
    if _RF is None:
        _RF = _autograd_function()
    meta = dict(N=int(g["N"]), sh_deg=int(g["sh_deg"]), C_o=int(g["C_o"]))
    r = _RF.apply(rast, meta, cams, g["mean"], g["quat"], g["log_scale"], g["opacity_logit"], g["mask_logit"],
                  g["sh"], g["sem"])
    return dict(zip(("rgb", "depth", "kmap", "normal", "sem", "T_final", "n_contrib"), r))
