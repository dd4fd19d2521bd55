"""ugs_prune_noalloc (the pruning compaction on the library's own scratch
array, for callers that cannot allocate device memory) gives exactly the
results of ugs_prune, which takes a caller scratch buffer, on two calls in a
row, the second on a smaller input, and refuses inputs above its limit."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _set(N, C_o, seed):
    import torch
    from paper_2510_12174_amd import scenes
    from paper_2510_12174_amd import unigs as U
    g_np, _, _ = scenes.make_scene(2, N=N, r=seed)
    g = U.to_device(g_np)
    if C_o != int(g["C_o"]):
        gen = torch.Generator(device="cuda").manual_seed(seed)
        g["sem"] = torch.randn(N, C_o, device="cuda", generator=gen)
        g["C_o"] = C_o
    gen = torch.Generator(device="cuda").manual_seed(100 + seed)
    states = [{k: torch.randn(g[k].shape, device="cuda", generator=gen) for k in U.PARAM_KEYS} for _ in range(2)]
    return g, states


def test_prune_noalloc_matches_prune():
    import torch
    from paper_2510_12174_amd import unigs as U
    if not torch.cuda.is_available():
        pytest.fail("GPU test needs a GPU")
    for N, C_o, T_k, seed in ((250_000, 32, 0.2, 1), (40_003, 12, 0.05, 2)):
        g, states = _set(N, C_o, seed)
        ref, ref_st, n_ref = U.prune(g, T_k, reset_k=True, states=states)
        got, got_st, n_got = U.prune(g, T_k, reset_k=True, states=states, noalloc=True)
        torch.cuda.synchronize()
        print(f"[noalloc] N={N} C_o={C_o} T_k={T_k}: kept {n_ref} / {n_got}", flush=True)
        assert n_got == n_ref and 0 < n_ref < N
        for k in U.PARAM_KEYS:
            assert torch.equal(got[k], ref[k]), k
            for a, b in zip(got_st, ref_st):
                assert torch.equal(a[k], b[k]), k


def test_prune_noalloc_limit():
    import ctypes as C
    import torch
    from paper_2510_12174_amd import unigs as U
    if not torch.cuda.is_available():
        pytest.fail("GPU test needs a GPU")
    N = U.UGS_PRUNE_NOALLOC_MAX_N + 1
    g = dict(N=N, sh_deg=0, C_o=0)
    for k, rows in (("mean", 3), ("quat", 4), ("log_scale", 3), ("opacity_logit", 1), ("mask_logit", 1), ("sh", 3)):
        g[k] = torch.zeros(rows * N, device="cuda")
    g["sem"] = torch.zeros(0, device="cuda")
    out = {k: torch.empty_like(g[k]) for k in U.PARAM_KEYS}
    nk = C.c_int64()
    rc = U.lib().ugs_prune_noalloc(C.byref(U.make_gaussians(g)), C.byref(U.make_grads(out)), 0, None, None, 0.2, 1,
                                   C.byref(nk), U._stream())
    assert rc == U.UGS_ERR_UNSUPPORTED
