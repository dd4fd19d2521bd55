"""Differentiable pruning on the GPU (ugs_prune, section 3.3): the compaction
against the oracle's reference, bit for bit, and the rendering of a pruned set
against the full set rendered with the pruning skip."""
import numpy as np
import pytest

from tests import harness as Hn

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def O():
    from oracle import oracle
    oracle.lib()
    return oracle


@pytest.mark.parametrize("T_k,reset", [(0.2, True), (0.05, False), (1.0, True)])
def test_prune_matches_reference(O, T_k, reset):
    import torch
    from paper_2510_12174_amd import unigs as U
    g, cams, opts = Hn.small_workload("w5s")
    rng = np.random.default_rng(5)
    st_np = {k: rng.standard_normal(np.asarray(g[k]).shape).astype(np.float32) for k in ("mean", "quat", "sh", "sem")}
    gd = U.to_device(g)
    st = {k: (torch.from_numpy(v).cuda() if v is not None else None) for k, v in st_np.items()}
    res, (rst,), n = U.prune(gd, T_k, reset_k=reset, states=[st])
    torch.cuda.synchronize()
    ref, (rref,), keep, amb = O.prune(g, T_k, reset=reset, states=[st_np])
    Hn.say(f"[prune T_k={T_k}] kept {n} of {g['N']} (reference {ref['N']}, ambiguous {int(amb.sum())})")
    assert not amb.any()
    assert n == ref["N"]
    for k in U.PARAM_KEYS:
        assert np.array_equal(res[k].cpu().numpy(), ref[k]), k
    for k in ("mean", "quat", "sh", "sem"):
        assert np.array_equal(rst[k].cpu().numpy(), rref[k]), k
    assert rst["log_scale"] is None


def test_pruned_set_renders_like_the_skip(O):
    """Rendering the pruned set (no reset, no skip) equals rendering the full
    set with the pruning skip at the same threshold, bit for bit."""
    import torch
    from paper_2510_12174_amd import unigs as U
    g, cams, opts = Hn.small_workload("w5s")
    T_k = float(opts["prune_Tk"])
    assert T_k > 0
    full, _, _ = Hn.gpu_run(g, cams, opts)
    gd = U.to_device(g)
    res, _, n = U.prune(gd, T_k, reset_k=False)
    torch.cuda.synchronize()
    assert 0 < n < g["N"]
    pruned_np = {k: (res[k].cpu().numpy() if k not in ("N", "sh_deg", "C_o") else res[k]) for k in res}
    part, _, _ = Hn.gpu_run(pruned_np, cams, dict(opts, prune_Tk=0.0))
    for x, y in zip(full, part):
        for k in ("rgb", "depth", "kmap", "normal", "sem", "T_final"):
            assert np.array_equal(x[k], y[k]), k
