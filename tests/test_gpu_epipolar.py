"""GPU parity of the epipolar verification and static recovery (Sec. IV-C,
Eq. (18)-(19)) through the C ABI against the FP64 oracle: distances, medians,
states and the restored MP, on ragged segments (empty, one match, either side
of a wave's 64, thousands), duplicate and invalid candidates, a pair without
baseline, and the candidates of a 1M-Gaussian map."""

import numpy as np
import pytest
import torch

from oracle import epipolar as ep
from paper_2602_21644_amd import gs, synth
from tests.gpu_util import torch_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return gs.Context(0)


def _run(ctx, cam1, cam2, p1, p2, ids, seg, mp, **kw):
    n = mp.size
    views = gs.ViewBatch([cam1, cam2], n)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    m, K = p1.shape[1], ids.size
    d = torch.full((max(m, 1),), -1.0, device="cuda")
    dbar = torch.full((max(K, 1),), -1.0, device="cuda")
    state = torch.full((max(K, 1),), 255, dtype=torch.uint8, device="cuda")
    mpd = dev(mp.astype(np.float32))
    gs.gs_epipolar_verify(ctx, views.s, 0, 1, dev(p1.astype(np.float32)), dev(p2.astype(np.float32)),
                          dev(ids.astype(np.int32)), dev(seg.astype(np.int64)), mpd, d, dbar, state, **kw)
    torch.cuda.synchronize()
    return torch_np(d)[:m], torch_np(dbar)[:K], torch_np(state)[:K], torch_np(mpd)


def _compare(got, ref, seg, eps):
    d, dbar, state, mp = got
    # distances: float32 from double on both sides; NaN canonical on the GPU;
    # written for the matches of valid candidates (the others keep the -1 fill)
    cov = np.zeros(d.size, bool)
    for k in range(state.size):
        if state[k] != ep.INVALID:
            cov[seg[k]:seg[k + 1]] = True
    assert np.all(d[~cov] == -1.0)
    nan = np.isnan(ref["d"]) & cov
    np.testing.assert_array_equal(np.isnan(d), nan)
    assert np.all(d.view(np.uint32)[nan] == ep.QNAN_BITS)
    ok = cov & ~nan
    np.testing.assert_allclose(d[ok], ref["d"][ok], rtol=3e-7, atol=0)
    # the kernel's median is the lower median of its own distances, exactly
    for k in range(dbar.size):
        b, e = seg[k], seg[k + 1]
        if state[k] in (ep.NO_MATCHES, ep.INVALID):
            assert np.isnan(dbar[k]) and state[k] == ref["state"][k]
            continue
        assert dbar[k].view(np.uint32) == ep.lower_median_f32(d[b:e]).view(np.uint32), k
    np.testing.assert_allclose(dbar, ref["dbar"], rtol=3e-7, atol=0, equal_nan=True)
    # decisions: identical away from the threshold
    border = np.abs(ref["dbar"].astype(np.float64) - eps) <= 1e-6 * max(eps, 1.0)
    np.testing.assert_array_equal(state[~border], ref["state"][~border])
    changed = np.zeros(mp.size, bool)
    changed[np.asarray(ref["_ids"])[border & (ref["state"] != ep.INVALID)]] = True
    np.testing.assert_array_equal(mp[~changed], ref["mp"][~changed])


def _ragged_case(seed=3):
    c = synth.epipolar_case(seed, 50000, 640, 480, 1200, per=(0, 40))
    p1, p2, seg, ids = c["p1"], c["p2"], c["seg"], c["ids"]
    m = p1.shape[1]
    rng = np.random.default_rng(seed)
    # extra candidates: segment lengths around the wave width and long ones
    # drawn from the existing matches (of static and moving Gaussians alike)
    extra_len = [1, 2, 63, 64, 65, 127, 128, 129, 500, 5000, 20000]
    src = rng.integers(0, m, sum(extra_len))
    p1 = np.concatenate([p1, p1[:, src]], axis=1)
    p2 = np.concatenate([p2, p2[:, src]], axis=1)
    seg = np.concatenate([seg, seg[-1] + np.cumsum(extra_len)])
    extra_ids = rng.choice(np.nonzero(c["mp"] > 0.5)[0], size=len(extra_len), replace=False)
    ids = np.concatenate([ids, extra_ids, ids[:5]]).astype(np.int32)  # five listed twice
    # the duplicates reuse their first segments
    seg = np.concatenate([seg, seg[-1] + np.cumsum(np.diff(c["seg"][:6]))])
    p1 = np.concatenate([p1, c["p1"][:, :c["seg"][5]]], axis=1)
    p2 = np.concatenate([p2, c["p2"][:, :c["seg"][5]]], axis=1)
    return c, p1, p2, ids, seg


def test_epipolar_ragged_parity(ctx):
    c, p1, p2, ids, seg = _ragged_case()
    for eps, tau, rest in ((1.0, 0.5, 0.0), (2.5, 0.7, 0.25)):
        got = _run(ctx, c["cam1"], c["cam2"], p1, p2, ids, seg, c["mp"], eps=eps, tau=tau, mp_restore=rest)
        ref = ep.verify(c["cam1"], c["cam2"], p1, p2, ids, seg, c["mp"], eps=eps, tau=tau, mp_restore=rest)
        ref["_ids"] = ids
        _compare(got, ref, seg, eps)
        st = got[2]
        print(f"\n[epipolar] eps {eps}: states {np.bincount(st, minlength=5).tolist()}")
        assert (st == ep.RESTORED).sum() > 50 and (st == ep.KEPT).sum() > 50 and (st == ep.NO_MATCHES).sum() > 0


def test_epipolar_invalid_candidates(ctx):
    """Ids out of range and match ranges outside [0, m] or reversed are
    reported INVALID and leave MP alone; the valid neighbours still agree."""
    c = synth.epipolar_case(4, 20000, 320, 240, 300, per=(1, 10))
    p1, p2, ids, seg = c["p1"], c["p2"], c["ids"].copy(), c["seg"].copy()
    m, n = p1.shape[1], c["mp"].size
    ids[3] = n
    ids[7] = -1
    seg_bad = seg.copy()
    seg_bad[11] = seg_bad[12] + 1  # candidate 11 reversed (and 10 ends past its start: still a valid range)
    seg_bad[-1] = m + 5  # the last range runs past m
    got = _run(ctx, c["cam1"], c["cam2"], p1, p2, ids, seg_bad, c["mp"])
    ref = ep.verify(c["cam1"], c["cam2"], p1, p2, ids, seg_bad, c["mp"])
    ref["_ids"] = np.clip(ids, 0, n - 1)
    assert got[2][3] == ep.INVALID and got[2][7] == ep.INVALID and got[2][11] == ep.INVALID
    assert got[2][-1] == ep.INVALID
    # the valid candidates' distances, medians, states and MP still agree
    _compare(got, ref, seg_bad, 1.0)


def test_epipolar_without_baseline(ctx):
    """Frames at one pose: F = 0, every distance is the quiet NaN, nothing is
    restored."""
    c = synth.epipolar_case(6, 20000, 320, 240, 200)
    got = _run(ctx, c["cam1"], c["cam1"], c["p1"], c["p2"], c["ids"], c["seg"], c["mp"])
    assert np.all(got[0].view(np.uint32) == ep.QNAN_BITS)
    assert not np.any(got[2] == ep.RESTORED)
    np.testing.assert_array_equal(got[3], c["mp"])


def test_epipolar_full_map(ctx):
    """50k candidates of a 1M-Gaussian map, about 16 matches each."""
    c = synth.epipolar_case(7, 1_000_000, 640, 480, 50000, per=(4, 28))
    got = _run(ctx, c["cam1"], c["cam2"], c["p1"], c["p2"], c["ids"], c["seg"], c["mp"])
    ref = ep.verify(c["cam1"], c["cam2"], c["p1"], c["p2"], c["ids"], c["seg"], c["mp"])
    ref["_ids"] = c["ids"]
    _compare(got, ref, c["seg"], 1.0)
    dyn = c["dynamic"][c["ids"]]
    sup_static = ~dyn & (c["mp"][c["ids"]] > 0.5)
    print(f"\n[epipolar 1M] {c['p1'].shape[1]} matches; restored {np.mean(got[2][sup_static] == 1):.3f} of the "
          f"suppressed static candidates, {np.mean(got[2][dyn] == 1):.3f} of the moving ones")
    assert np.mean(got[2][sup_static] == ep.RESTORED) > 0.9
