"""The synthetic ablation runner on the GPU (tracking, epipolar verification,
scheduler and MP update per frame): refresh counts of the three scheduling
policies, exact lists, tracked poses close to the truth, and the variants'
metrics in range. The numbers themselves are reported, not pinned."""

import math

import pytest
import torch

from paper_2602_21644_amd import gs, sequence, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return gs.Context(0)


@pytest.fixture(scope="module")
def seq():
    return synth.box_sequence(41, 40000, 160, 120, 24, box_frac=0.1, zmin=1.5, zmax=5.0)


def test_scheduling_policies(ctx, seq):
    res = {v: sequence.run(ctx, seq, v, track_iters=15, k_cand=800) for v in
           ("always", "fixed_interval", "adaptive", "instant", "ins_only", "geo_only", "no_recovery")}
    for r in res.values():
        print(f"\n[ablation] {r}")
        assert r["exact"]
        assert r["ate_cm"] < 2.0 and r["rot_err_deg"] < 0.5
        assert 0.0 <= r["mp_abs_error"] < 0.6
    F = res["always"]["frames"]
    assert res["always"]["refreshes"] == F
    assert res["fixed_interval"]["refreshes"] == math.ceil(F / 10)
    assert math.ceil(F / 10) <= res["adaptive"]["refreshes"] <= F
    assert res["adaptive"]["restored"] > 0 and res["no_recovery"]["restored"] == 0
    assert res["adaptive"]["label_error_pct"] < 50.0
