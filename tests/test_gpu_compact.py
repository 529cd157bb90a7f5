"""gs_compact through the C ABI against the oracle's removal by a drop mask:
bit-exact planes, kept count and scene offsets, on ragged sizes, empty and
full masks, repeated and empty scenes, the plane limit and more tiles than
one scan chunk holds."""

import numpy as np
import pytest
import torch

from paper_2602_21644_amd import gs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return gs.Context(0)


def _run(ctx, n, n_planes, p_drop, seg, seed):
    rng = np.random.default_rng(seed)
    drop = (rng.random(n) < p_drop).astype(np.uint8)
    src = [rng.normal(size=n).astype(np.float32) for _ in range(n_planes)]
    d_drop = torch.from_numpy(drop).cuda()
    d_src = [torch.from_numpy(x).cuda() for x in src]
    d_dst = [torch.full((max(n, 1),), float("nan"), device="cuda") for _ in range(n_planes)]
    n_out = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    seg_out = torch.full((len(seg),), -1, dtype=torch.int64, device="cuda") if seg is not None else None
    ws = torch.empty(gs.gs_workspace_size(ctx, None, gs.GS_OP_COMPACT, n), dtype=torch.uint8, device="cuda")
    gs.gs_compact(ctx, d_drop, d_src, d_dst, n_out, ws, seg_begin=seg, seg_out=seg_out)
    torch.cuda.synchronize()
    import oracle
    ref, off = oracle.compact(src, drop.astype(bool), seg)
    k = int(n_out.item())
    assert k == ref[0].size if n_planes else k == int((drop == 0).sum())
    for got, want in zip(d_dst, ref):
        np.testing.assert_array_equal(got[:k].cpu().numpy(), want)
        if k < n:  # nothing written beyond the kept count
            assert torch.isnan(got[k:]).all()
    if seg is not None:
        assert seg_out.cpu().tolist() == off.tolist()


@pytest.mark.parametrize("n,n_planes,p_drop,seg", [
    (0, 3, 0.5, [0, 0]), (1, 1, 0.0, [0, 1]), (1, 1, 1.0, [0, 1]), (2047, 17, 0.3, None),
    (2048, 17, 0.3, [0, 1000, 1000, 2048]), (100_003, 64, 0.1, [0, 5, 2048, 4096, 50_000, 100_003]),
    (1_000_000, 17, 0.02, [0, 1_000_000]), (1_000_000, 2, 1.0, [0, 600_000, 1_000_000]),
    (1_000_000, 2, 0.0, [0, 999_999, 1_000_000]), (2_500_001, 3, 0.5, [0, 2_097_152, 2_500_001])])
def test_compact_matches_oracle(ctx, orc, n, n_planes, p_drop, seg):
    _run(ctx, n, n_planes, p_drop, seg, seed=n + n_planes)


def test_compact_rejects_bad_arguments(ctx):
    n = 1000
    drop = torch.zeros(n, dtype=torch.uint8, device="cuda")
    a = torch.zeros(n, device="cuda")
    n_out = torch.zeros(1, dtype=torch.int64, device="cuda")
    ws = torch.empty(gs.gs_workspace_size(ctx, None, gs.GS_OP_COMPACT, n), dtype=torch.uint8, device="cuda")
    with pytest.raises(gs.GSError, match="overlap"):
        gs.gs_compact(ctx, drop, [a], [a], n_out, ws)
    with pytest.raises(gs.GSError, match="seg_begin"):
        gs.gs_compact(ctx, drop, [a], [torch.zeros(n, device="cuda")], n_out, ws, seg_begin=[0, 10],
                      seg_out=torch.zeros(2, dtype=torch.int64, device="cuda"))
    many = [torch.zeros(n, device="cuda") for _ in range(gs.GS_COMPACT_MAX_PLANES + 1)]
    outs = [torch.zeros(n, device="cuda") for _ in range(gs.GS_COMPACT_MAX_PLANES + 1)]
    with pytest.raises(gs.GSError, match="planes"):
        gs.gs_compact(ctx, drop, many, outs, n_out, ws)
