"""The C-ABI library loads, exports every symbol include/unigs.h declares, and
rejects invalid arguments before touching the GPU.  CPU only."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def U():
    from paper_2510_12174_amd import unigs
    if not os.path.exists(unigs.LIB):
        from paper_2510_12174_amd import build
        build.build()
    unigs.lib()
    return unigs


def header_functions():
    src = open(os.path.join(ROOT, "include", "unigs.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ugs_[a-z_]+)\s*\(", src)))


def test_exports_match_header(U):
    names = header_functions()
    assert len(names) >= 18
    L = U.lib()
    for n in names:
        assert hasattr(L, n), n
    assert sorted(U.EXPORTS) == names


def test_symbols_are_exported_dynamically(U):
    import subprocess
    out = subprocess.run(["nm", "-D", "--defined-only", U.LIB], capture_output=True, text=True).stdout
    for n in header_functions():
        assert re.search(rf"\bT {n}\b", out), n


def test_options_validation(U):
    L = U.lib()
    ctx = C.c_void_p()
    o = U.default_options()
    assert (o.tile_w, o.tile_h, o.step1, o.step2, o.orient_sign) == (16, 16, 1, 2, 1)
    assert L.ugs_create(C.byref(ctx), C.byref(o)) == U.UGS_OK
    bad = U.default_options(tile_w=12)
    assert L.ugs_set_options(ctx, C.byref(bad)) == U.UGS_ERR_UNSUPPORTED
    bad = U.default_options(orient_sign=0)
    assert L.ugs_set_options(ctx, C.byref(bad)) == U.UGS_ERR_INVALID_ARG
    bad = U.default_options(lambda_=1.5)
    assert L.ugs_set_options(ctx, C.byref(bad)) == U.UGS_ERR_INVALID_ARG
    bad = U.default_options(half_outputs=2)
    assert L.ugs_set_options(ctx, C.byref(bad)) == U.UGS_ERR_INVALID_ARG
    bad = U.default_options(depth_mode=3)
    assert L.ugs_set_options(ctx, C.byref(bad)) == U.UGS_ERR_INVALID_ARG
    assert o.depth_mode == 0
    for m in (1, 2):
        ok = U.default_options(depth_mode=m)
        assert L.ugs_set_options(ctx, C.byref(ok)) == U.UGS_OK
    for tw, th in ((8, 8), (32, 8), (16, 16)):
        ok = U.default_options(tile_w=tw, tile_h=th)
        assert L.ugs_set_options(ctx, C.byref(ok)) == U.UGS_OK
    L.ugs_destroy(ctx)


def _cams():
    from paper_2510_12174_amd import scenes
    return U_cams([scenes.camera(64, 48, 50, 50, 32, 24, np.eye(3), [0, 0, 3])])


def U_cams(cams):
    from paper_2510_12174_amd import unigs
    return unigs.make_cameras(cams)


def test_workspace_size_and_limits(U):
    L = U.lib()
    ctx = C.c_void_p()
    assert L.ugs_create(C.byref(ctx), None) == U.UGS_OK
    cams = _cams()
    n = C.c_size_t()
    assert L.ugs_workspace_size(ctx, 1000, 8, 3, cams, 1, 100000, C.byref(n)) == U.UGS_OK
    small = n.value
    assert L.ugs_workspace_size(ctx, 1000, 8, 3, cams, 1, 200000, C.byref(n)) == U.UGS_OK
    # 2 x 4 B keys + 2 x 4 B values per pair, plus 4 bits of activity mask
    assert abs((n.value - small) - 100000 * 16.5) <= 6 * 256
    assert L.ugs_workspace_size(ctx, 1000, 200, 3, cams, 1, 10, C.byref(n)) == U.UGS_OK
    assert L.ugs_workspace_size(ctx, 1000, 257, 3, cams, 1, 10, C.byref(n)) == U.UGS_ERR_UNSUPPORTED
    assert L.ugs_workspace_size(ctx, 1000, 8, 4, cams, 1, 10, C.byref(n)) == U.UGS_ERR_UNSUPPORTED
    assert L.ugs_workspace_size(ctx, -1, 8, 3, cams, 1, 10, C.byref(n)) == U.UGS_ERR_INVALID_ARG
    assert L.ugs_workspace_size(ctx, 10, 8, 3, cams, 0, 10, C.byref(n)) == U.UGS_ERR_INVALID_ARG
    assert L.ugs_workspace_size(ctx, 10, 8, 3, cams, 1, 1 << 40, C.byref(n)) == U.UGS_ERR_INVALID_ARG
    badcam = _cams()
    badcam[0].fx = 0.0
    assert L.ugs_workspace_size(ctx, 10, 8, 3, badcam, 1, 10, C.byref(n)) == U.UGS_ERR_INVALID_ARG
    L.ugs_destroy(ctx)


def test_calls_rejected_before_launch(U):
    """Null / inconsistent arguments and out-of-order calls return status codes
    without any HIP call (this runs on a machine without a GPU)."""
    L = U.lib()
    ctx = C.c_void_p()
    assert L.ugs_create(C.byref(ctx), None) == U.UGS_OK
    cams = _cams()
    g = U.ugs_gaussians()
    g.N, g.sh_deg, g.C_o = 10, 0, 4  # null parameter pointers
    assert L.ugs_project(ctx, C.byref(g), cams, 1, C.c_void_p(256), 1 << 20, None) == U.UGS_ERR_INVALID_ARG
    g.sh_deg = 5
    assert L.ugs_project(ctx, C.byref(g), cams, 1, C.c_void_p(256), 1 << 20, None) == U.UGS_ERR_UNSUPPORTED
    assert L.ugs_bin_sort(ctx, C.c_void_p(256), None, None) == U.UGS_ERR_STATE
    assert L.ugs_render_fwd(ctx, C.byref(g), C.c_void_p(256), None, None) == U.UGS_ERR_STATE
    assert L.ugs_step_replay(ctx, None) == U.UGS_ERR_NOT_CAPTURED
    assert L.ugs_bin_sort(None, None, None, None) == U.UGS_ERR_INVALID_ARG
    assert L.ugs_time_stage(ctx, 9, None, None) == U.UGS_ERR_INVALID_ARG
    assert L.ugs_time_stage(ctx, 0, None, None) == U.UGS_OK
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert L.ugs_status_string(code)
    L.ugs_destroy(ctx)


def test_prune_rejections(U):
    """ugs_prune validates before touching the device."""
    L = U.lib()
    nb = C.c_size_t()
    assert L.ugs_prune_scratch_size(1000, C.byref(nb)) == U.UGS_OK and nb.value >= 8000
    assert L.ugs_prune_scratch_size(-1, C.byref(nb)) == U.UGS_ERR_INVALID_ARG
    g = U.ugs_gaussians()
    g.N, g.sh_deg, g.C_o = 10, 0, 0
    g.mask_logit = 256
    out = U.ugs_gaussian_grads()
    n = C.c_int64()
    # NULL parameter set, NULL count, negative threshold, missing scratch
    assert L.ugs_prune(None, C.byref(out), 0, None, None, 0.2, 1, C.c_void_p(256), 4096, C.byref(n), None) \
        == U.UGS_ERR_INVALID_ARG
    assert L.ugs_prune(C.byref(g), C.byref(out), 0, None, None, 0.2, 1, C.c_void_p(256), 4096, None, None) \
        == U.UGS_ERR_INVALID_ARG
    assert L.ugs_prune(C.byref(g), C.byref(out), 0, None, None, -0.1, 1, C.c_void_p(256), 4096, C.byref(n), None) \
        == U.UGS_ERR_INVALID_ARG
    assert L.ugs_prune(C.byref(g), C.byref(out), 0, None, None, 0.2, 1, None, 4096, C.byref(n), None) \
        == U.UGS_ERR_INVALID_ARG
    # scratch too small, state sets announced but missing
    assert L.ugs_prune(C.byref(g), C.byref(out), 0, None, None, 0.2, 1, C.c_void_p(256), 8, C.byref(n), None) \
        == U.UGS_ERR_INVALID_ARG
    assert L.ugs_prune(C.byref(g), C.byref(out), 2, None, None, 0.2, 1, C.c_void_p(256), 4096, C.byref(n), None) \
        == U.UGS_ERR_INVALID_ARG


def test_loss_rejections(U):
    """ugs_loss validates before touching the device."""
    L = U.lib()
    nb = C.c_size_t()
    cams = U.make_cameras([dict(W=64, H=48, fx=50, fy=50, cx=32, cy=24, R=np.eye(3), t=np.zeros(3))])
    assert L.ugs_loss_scratch_size(cams, 1, C.byref(nb)) == U.UGS_OK and nb.value >= 36 * 64 * 48
    assert L.ugs_loss_scratch_size(cams, 0, C.byref(nb)) == U.UGS_ERR_INVALID_ARG
    o = U.loss_options()
    assert abs(o.lambda_[0] - 1.0) < 1e-7 and abs(o.lambda_[5] - 0.1) < 1e-7 and o.balance == 1
    out, gt, up = U.ugs_outputs(), U.ugs_targets(), U.ugs_upstream()
    for s in (out, gt, up):
        for f, _ in s._fields_:
            setattr(s, f, 256)
    sc = C.c_void_p(256)
    ok = lambda **kw: L.ugs_loss(cams, 1, kw.get("C_o", 4), C.byref(out), C.byref(gt), C.byref(o), C.byref(up),
                                 C.c_void_p(256), kw.get("sc", sc), kw.get("nb", nb.value), None)
    assert ok(nb=8) == U.UGS_ERR_INVALID_ARG             # scratch too small
    assert ok(sc=C.c_void_p(260)) == U.UGS_ERR_INVALID_ARG  # misaligned scratch
    assert ok(C_o=0) == U.UGS_ERR_INVALID_ARG             # labels without channels
    assert ok(C_o=U.UGS_MAX_CHANNELS + 1) == U.UGS_ERR_INVALID_ARG
    gt.rgb = None
    assert ok() == U.UGS_ERR_INVALID_ARG
    gt.rgb = 256
    out.kmap = 258
    assert ok() == U.UGS_ERR_INVALID_ARG                  # misaligned map


def test_plain_c_program_links_the_abi(U, tmp_path):
    """The header is plain C99 and a C program links the library and calls its
    host-side entry points (defaults, status strings, argument rejection)."""
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "abi.c"
    src.write_text(r'''
#include <stdio.h>
#include "unigs.h"
int main(void) {
    ugs_options o;
    ugs_default_options(&o);
    ugs_loss_options lo;
    ugs_default_loss_options(&lo);
    size_t nb = 0;
    int bad = ugs_prune_scratch_size(-1, &nb);
    printf("%d %d %d %.2f %d %s\n", o.tile_w, o.tile_h, o.depth_mode, lo.lambda[1], bad,
           ugs_status_string(UGS_ERR_CAPACITY));
    return 0;
}
''')
    exe = tmp_path / "abi"
    libdir = os.path.dirname(U.LIB)
    subprocess.check_call([gcc, "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"), str(src),
                           "-o", str(exe), "-L", libdir, "-lunigs", "-Wl,-rpath," + libdir])
    out = subprocess.check_output([str(exe)], text=True).split()
    assert out[:5] == ["16", "16", "0", "0.10", str(U.UGS_ERR_INVALID_ARG)]
    assert "capacity" in " ".join(out[5:]).lower()


def test_binding_validates_maps(U):
    """The binding refuses maps it would hand to the C ABI with the wrong element
    type, device, layout or size (CPU tensors: the dtype check comes first)."""
    import torch
    with pytest.raises(ValueError, match="dtype"):
        U.check_map(torch.zeros(16, dtype=torch.int64), "gt label", torch.int32, 16)
    with pytest.raises(ValueError, match="dtype"):
        U.check_map(torch.zeros(16, dtype=torch.float64), "gt rgb", torch.float32, 16)
    with pytest.raises(ValueError, match="CUDA"):
        U.check_map(torch.zeros(16, dtype=torch.int32), "gt label", torch.int32, 16)
    with pytest.raises(ValueError, match="tensor"):
        U.check_map(np.zeros(16, np.int32), "gt label", torch.int32, 16)
    with pytest.raises(ValueError, match="dtype"):
        U.check_upstream(dict(sem_label=torch.zeros(4, dtype=torch.int64)), 4, 2)
