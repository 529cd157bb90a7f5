"""Pins of the FP64 reference of the epipolar verification (Sec. IV-C, Eq.
(18)-(19)), CPU only: the epipoles are F's null vectors, F matches the
textbook construction from projection matrices, exact matches have distance
0, a move across the epipolar line by delta pixels has distance delta, the
lower median against brute-force sorting, and the restore rule on hand-built
cases."""

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from oracle import epipolar as ep
from paper_2602_21644_amd import synth


def _cams(seed, W=640, H=480, trans=0.1, deg=5.0):
    rng = np.random.default_rng(seed)
    cams = []
    for _ in range(2):
        c = synth.camera(W, H)
        R = Rotation.from_rotvec(rng.normal(size=3) * np.deg2rad(deg)).as_matrix()
        c["T_cw"] = np.concatenate([R, rng.normal(size=(3, 1)) * trans], axis=1)  # float64, orthonormal
        cams.append(c)
    return cams


def _project(cam, X):
    T = np.asarray(cam["T_cw"], dtype=np.float64)
    Xc = T[:, :3] @ X + T[:, 3:4]
    return np.stack([cam["fx"] * Xc[0] / Xc[2] + cam["cx"], cam["fy"] * Xc[1] / Xc[2] + cam["cy"]])


def _centre(cam):
    T = np.asarray(cam["T_cw"], dtype=np.float64)
    return -T[:, :3].T @ T[:, 3]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_epipoles_are_null_vectors(seed):
    """F e1 = 0 and F^T e2 = 0 for e1 the image of camera 2's centre in frame 1
    and e2 the image of camera 1's centre in frame 2."""
    c1, c2 = _cams(seed)
    F = ep.fundamental(c1, c2)
    e1 = np.append(_project(c1, _centre(c2)[:, None])[:, 0], 1.0)
    e2 = np.append(_project(c2, _centre(c1)[:, None])[:, 0], 1.0)
    scale = np.abs(F).max()
    assert np.abs(F @ e1).max() < 1e-12 * scale * np.abs(e1).max()
    assert np.abs(F.T @ e2).max() < 1e-12 * scale * np.abs(e2).max()


@pytest.mark.parametrize("seed", [3, 4])
def test_fundamental_matches_projection_matrix_construction(seed):
    """Up to scale, F = [e2]_x P2 P1^+ with P = K [R | t] and e2 = P2 C1."""
    c1, c2 = _cams(seed)
    P = [ep.intrinsic_matrix(c) @ np.asarray(c["T_cw"], dtype=np.float64) for c in (c1, c2)]
    e2 = P[1] @ np.append(_centre(c1), 1.0)
    Fh = ep.skew(e2) @ P[1] @ np.linalg.pinv(P[0])
    F = ep.fundamental(c1, c2)
    a, b = F / np.linalg.norm(F), Fh / np.linalg.norm(Fh)
    if np.sum(a * b) < 0:
        b = -b
    np.testing.assert_allclose(a, b, atol=1e-9)


def test_exact_matches_have_zero_distance():
    c1, c2 = _cams(5)
    rng = np.random.default_rng(6)
    X = np.stack([rng.uniform(-1, 1, 500), rng.uniform(-1, 1, 500), rng.uniform(1.0, 6.0, 500)])
    d = ep.epipolar_distance(ep.fundamental(c1, c2), _project(c1, X), _project(c2, X))
    assert np.abs(d).max() < 1e-8


def test_distance_across_the_line_is_the_offset():
    """Moving p2 by delta along the unit normal (a, b) / |(a, b)| of its
    epipolar line gives distance delta; moving it along the line gives 0."""
    c1, c2 = _cams(7)
    rng = np.random.default_rng(8)
    X = np.stack([rng.uniform(-1, 1, 200), rng.uniform(-1, 1, 200), rng.uniform(1.0, 6.0, 200)])
    p1, p2 = _project(c1, X), _project(c2, X)
    F = ep.fundamental(c1, c2)
    line = F @ np.vstack([p1, np.ones(200)])
    nrm = line[:2] / np.hypot(line[0], line[1])
    delta = rng.uniform(0.0, 30.0, 200)
    np.testing.assert_allclose(ep.epipolar_distance(F, p1, p2 + delta * nrm), delta, atol=1e-7)
    along = np.stack([-nrm[1], nrm[0]]) * rng.uniform(-50, 50, 200)
    assert np.abs(ep.epipolar_distance(F, p1, p2 + along)).max() < 1e-7


def test_pure_rotation_is_degenerate():
    """Without translation (below 1e-6) F = 0: every distance is NaN and
    nothing is restored; a float32 copy of the rotated pose is degenerate too."""
    c1, _ = _cams(9)
    c2 = dict(c1)
    R = Rotation.from_rotvec([0.01, -0.02, 0.005]).as_matrix()
    T1 = np.asarray(c1["T_cw"], dtype=np.float64)
    c2["T_cw"] = np.concatenate([R @ T1[:, :3], (R @ T1[:, 3])[:, None]], axis=1)
    assert np.abs(ep.fundamental(c1, c2)).max() < 1e-15
    p = np.array([[100.0, 200.0], [50.0, 60.0]])
    r = ep.verify(c1, c2, p, p, [0], [0, 2], np.array([0.9], np.float32))
    assert np.isnan(r["dbar"][0]) and r["state"][0] == ep.KEPT and r["mp"][0] == np.float32(0.9)
    assert np.all(r["d"].view(np.uint32) == ep.QNAN_BITS)
    c3 = dict(c2, T_cw=np.asarray(c2["T_cw"], np.float32))
    c1f = dict(c1, T_cw=np.asarray(c1["T_cw"], np.float32))
    assert np.abs(ep.fundamental(c1f, c3)).max() == 0.0
    # just above the limit the pair is usable
    c4 = dict(c2, T_cw=c2["T_cw"] + np.array([[0, 0, 0, 2e-6]] * 3))
    assert np.abs(ep.fundamental(c1, c4)).max() > 0


def test_lower_median_against_sorting():
    rng = np.random.default_rng(10)
    for n in list(range(1, 12)) + [64, 65, 1000]:
        x = rng.uniform(0, 5, n).astype(np.float32)
        assert ep.lower_median_f32(x) == np.sort(x)[(n - 1) // 2]
    x = np.array([np.inf, 1.0, np.nan, 2.0], np.float32)  # order: 1, 2, inf, NaN
    assert ep.lower_median_f32(ep.to_f32_canonical(x)) == np.float32(2.0)
    x = np.array([np.nan, np.nan, 3.0], np.float32)
    assert np.isnan(ep.lower_median_f32(ep.to_f32_canonical(x)))
    assert np.isnan(ep.lower_median_f32(np.zeros(0, np.float32)))
    # a negative NaN from the arithmetic counts as the positive quiet NaN
    neg = np.array([0x7FC00000 | 0x80000000], np.uint32).view(np.float32)
    assert ep.to_f32_canonical(neg).view(np.uint32)[0] == ep.QNAN_BITS


def _line_case(offsets):
    """One candidate per offset list: matches moved across their epipolar
    lines by the given offsets (pixels)."""
    c1, c2 = _cams(11)
    rng = np.random.default_rng(12)
    p1s, p2s, seg = [], [], [0]
    F = ep.fundamental(c1, c2)
    for offs in offsets:
        k = len(offs)
        X = np.stack([rng.uniform(-1, 1, k), rng.uniform(-1, 1, k), rng.uniform(1.0, 6.0, k)])
        p1, p2 = _project(c1, X), _project(c2, X)
        line = F @ np.vstack([p1, np.ones(k)])
        p2 = p2 + np.asarray(offs) * line[:2] / np.hypot(line[0], line[1])
        p1s.append(p1)
        p2s.append(p2)
        seg.append(seg[-1] + k)
    return c1, c2, np.concatenate(p1s, axis=1), np.concatenate(p2s, axis=1), np.array(seg)


def test_restore_rule_hand_built():
    """Lower median of {0.2, 3, 0.4, 5} is 0.4 < 1: restored when suppressed;
    a median of exactly-epsilon-ish 1.5 stays; MP at tau is not suppressed;
    no matches keep the MP; an out-of-range id is invalid."""
    offs = [[0.2, 3.0, 0.4, 5.0], [1.5, 2.0, 0.1], [0.0, 0.0], [], [0.1], [0.3, 0.3]]
    c1, c2, p1, p2, seg = _line_case(offs)
    ids = np.array([0, 1, 2, 3, 4, 99])
    mp = np.array([0.9, 0.9, 0.5, 0.9, 0.7], np.float32)
    r = ep.verify(c1, c2, p1, p2, ids, seg, mp, eps=1.0, tau=0.5, mp_restore=0.0)
    assert r["dbar"][0] == pytest.approx(0.4, abs=1e-5)
    assert r["dbar"][1] == pytest.approx(1.5, abs=1e-5)
    np.testing.assert_array_equal(r["state"], [ep.RESTORED, ep.KEPT, ep.NOT_SUPPRESSED, ep.NO_MATCHES,
                                               ep.RESTORED, ep.INVALID])
    np.testing.assert_array_equal(r["mp"], np.array([0.0, 0.9, 0.5, 0.9, 0.0], np.float32))
    # strict: a median equal to eps does not restore
    eps = float(r["dbar"][0])
    r2 = ep.verify(c1, c2, p1, p2, ids[:1], seg[:2], mp, eps=eps)
    assert r2["state"][0] == ep.KEPT
    r3 = ep.verify(c1, c2, p1, p2, ids[:1], seg[:2], mp, eps=np.nextafter(np.float32(eps), np.float32(2)))
    assert r3["state"][0] == ep.RESTORED


def test_synthetic_case_separates_static_from_moving():
    """On the generated two-keyframe case most static Gaussians that MP
    suppresses are restored and few moving ones are."""
    c = synth.epipolar_case(5, 100000, 640, 480, 3000)
    r = ep.verify(c["cam1"], c["cam2"], c["p1"], c["p2"], c["ids"], c["seg"], c["mp"])
    dyn = c["dynamic"][c["ids"]]
    sup_static = ~dyn & (c["mp"][c["ids"]] > 0.5) & (np.diff(c["seg"]) > 0)
    assert np.mean(r["state"][sup_static] == ep.RESTORED) > 0.9
    assert np.mean(r["state"][dyn] == ep.RESTORED) < 0.15
