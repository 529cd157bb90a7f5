"""Pins of the semantic-on-demand scheduler reference (Sec. IV-B, Eq.
(13)-(17)), CPU only, and the library's host-side scheduler (gs_sched_decide,
no GPU needed) against it."""

import numpy as np
import pytest

from oracle import scheduler as osch


def _refresh_frames(sch, U, E, frames):
    return [t for t in range(frames) if sch.decide(U(t), E(t))]


def test_max_skip_alone_refreshes_every_n_max():
    """S never above theta: the first frame and every N_max-th after it."""
    sch = osch.Scheduler()
    assert _refresh_frames(sch, lambda t: 0.2, lambda t: 0.0, 35) == [0, 10, 20, 30]
    sch = osch.Scheduler(n_max=3)
    assert _refresh_frames(sch, lambda t: 0.0, lambda t: 0.0, 10) == [0, 3, 6, 9]


def test_score_above_theta_refreshes_and_restarts_the_count():
    sch = osch.Scheduler()
    assert _refresh_frames(sch, lambda t: 1.0 if t == 4 else 0.1, lambda t: 0.2 if t == 4 else 0.0,
                           30) == [0, 4, 14, 24]  # S = 0.5 + 0.05 at frame 4
    # U = 0.9 alone gives S = 0.45 < 0.5 at frame 4: it is R that tips it
    U = lambda t: 0.9 if t == 4 else 0.1
    assert _refresh_frames(osch.Scheduler(), U, lambda t: 0.0, 12) == [0, 10]
    sch = osch.Scheduler()
    E = lambda t: 1.0 if t == 4 else 0.0  # R = 0.5
    assert _refresh_frames(sch, U, E, 12) == [0, 4]
    assert sch.S == pytest.approx(0.5 * 0.1)


def test_theta_itself_does_not_trigger_and_R_saturates():
    """S = theta is no trigger (strict); R = clip(e_bar / e_ref, 0, 1) so
    with w_r = theta = 0.5 the inconsistency alone never triggers."""
    sch = osch.Scheduler()
    sch.decide(0.0, 0.0)  # the first frame
    assert not sch.decide(1.0, 0.0)  # S = 0.5
    assert not sch.decide(0.0, 1e9) and sch.R == 1.0 and sch.S == 0.5
    assert sch.decide(1e-3, 1e9)  # S = 0.5005
    assert osch.Scheduler(w_u=0.3, w_r=0.7).decide(0.0, 0.0)  # first frame
    s2 = osch.Scheduler(w_u=0.3, w_r=0.7)
    s2.decide(0, 0)
    assert s2.decide(0.0, 1.5) and s2.R == 0.75


def test_e_bar_uses_the_static_candidates_with_a_median():
    dbar = np.array([1.0, 3.0, np.nan, 10.0, 5.0], np.float32)
    state = np.array([2, 2, 2, 0, 2], np.uint8)  # 10.0 is a suppressed candidate
    assert osch.e_bar_of(dbar, state) == pytest.approx(3.0)
    assert osch.e_bar_of(dbar, np.zeros(5, np.uint8)) == 0.0
    assert osch.e_bar_of([], []) == 0.0


def test_sequence_reuses_stale_masks_with_the_slower_rate(orc):
    """Fixed policy, N = 3: frames 1 and 2 run on frame 0's masks with
    alpha' = rho alpha (Eq. (17)); frame 3 on its own masks at full rate."""
    from paper_2602_21644_amd import synth
    frames = synth.mp_sequence_inputs(3, 3000, 64, 48, 4)
    out = osch.run_mp_sequence(frames, policy="fixed", n_fixed=3)
    assert [o["refresh"] for o in out] == [True, False, False, True]
    mp = frames[0]["mp"]
    for t, o in enumerate(out):
        masks = frames[0 if t in (1, 2) else t]["instance_id"]
        inp = dict(frames[t], instance_id=masks, mp=mp)
        stale = orc.mp.mp_update(inp, seg_updated=t not in (1, 2))
        fresh = orc.mp.mp_update(inp, seg_updated=True)
        np.testing.assert_array_equal(o["result"]["mp"], stale["mp"])
        if t in (1, 2):
            np.testing.assert_allclose(stale["alpha"], 0.5 * fresh["alpha"], rtol=1e-12)
        mp = stale["mp"].astype(np.float32)


def test_library_scheduler_matches_reference():
    """gs_sched_decide (host code of the library) against the reference on
    random sequences: the same decisions, S within float32 rounding."""
    from paper_2602_21644_amd import gs
    rng = np.random.default_rng(0)
    for trial in range(20):
        kw = dict(w_u=float(rng.uniform(0, 1)), theta=float(rng.uniform(0.2, 0.8)), e_ref=float(rng.uniform(0.5, 4)),
                  n_max=int(rng.integers(1, 12)))
        kw["w_r"] = 1.0 - kw["w_u"]
        ref = osch.Scheduler(**kw)
        p = gs.sched_params(**kw)
        st = gs.sched_state(p)
        for t in range(40):
            U = float(rng.uniform(0, 1))
            k = int(rng.integers(0, 30))
            dbar = np.abs(rng.normal(0, rng.uniform(0.1, 5), k)).astype(np.float32)
            dbar[rng.random(k) < 0.1] = np.nan
            es = rng.integers(0, 5, k).astype(np.uint8)
            want = ref.decide(np.float32(U), osch.e_bar_of(dbar, es))
            got = gs.gs_sched_decide(p, st, U, dbar, es)
            if abs(ref.S - kw["theta"]) < 1e-5:
                break  # float32 and float64 scores may fall either side: end this sequence
            assert got == want, (trial, t)
            assert st.S == pytest.approx(ref.S, abs=1e-6) and st.e_bar == pytest.approx(ref.e_bar, rel=1e-6)
            assert st.n_refresh == ref.n_refresh and st.dt == ref.dt
    with pytest.raises(gs.GSError):
        gs.gs_sched_decide(gs.sched_params(w_u=0.6, w_r=0.6), gs.sched_state(gs.sched_params()), 0.0)
