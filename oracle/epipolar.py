"""FP64 reference of the epipolar verification and static recovery of
Sec. IV-C (Eq. (18)-(19), epsilon = 1 px from Sec. V-A).

TEST INFRASTRUCTURE ONLY (see the package docstring).

For a pair of frames with world->camera poses (R1, t1), (R2, t2) and pinhole
intrinsics K1, K2, the relative motion X2 = R X1 + t has R = R2 R1^T and
t = t2 - R t1; the essential matrix is E = [t]_x R and the fundamental matrix
F = K2^-T E K1^-1. A match (p1, p2) of pixels (u1, v1), (u2, v2) has the
epipolar line l2 = F [u1, v1, 1]^T = (a, b, c) in frame 2 and the distance
d = |[u2, v2, 1] l2| / sqrt(a^2 + b^2) (Eq. (18)).

Per candidate Gaussian G with matches M(G), d_bar(G) is the median of its
distances (Eq. (19)); G is consistent with static motion when d_bar < eps.
A candidate that MP suppresses and that passes the test is restored as
static. Readings (the paper leaves them open):
  * the distances are rounded to float32 (the precision the kernel stores
    them in) before the median; a NaN distance (a match on the epipole, or a
    pair without translation, where F = 0) counts as the positive quiet NaN,
    which orders above +inf;
  * the median of an even count is the lower median (as in the MP update),
    taken over the float32 values in the order of their bit patterns;
  * MP suppresses G when mp > tau (strict, the dynamic-label rule of
    Eq. (12)); restoring writes mp_restore (default 0, fully static) to G's
    MP; d_bar < eps is strict and a NaN d_bar never restores;
  * a candidate without matches keeps its MP (state NO_MATCHES), one whose id
    or match range is out of bounds is skipped (state INVALID);
  * a pair whose relative translation is shorter than T_MIN = 1e-6 (scene
    units, metres here) has no usable baseline: F is taken as 0, so every
    distance is NaN (the rounding residue of a pure rotation would otherwise
    give finite, meaningless distances).

Pinned by tests/test_oracle_epipolar.py: the null vectors of F are the
epipoles (each camera's centre seen by the other), F agrees up to scale with
the textbook construction [e2]_x P2 P1^+ from the projection matrices, exact
matches have d = 0, a match moved by delta pixels across its epipolar line
has d = delta, the lower median against brute-force sorting (with NaN and
inf), and the restore rule on hand-built cases.
"""

from __future__ import annotations

import numpy as np

KEPT, RESTORED, NOT_SUPPRESSED, NO_MATCHES, INVALID = 0, 1, 2, 3, 4
QNAN_BITS = np.uint32(0x7FC00000)
T_MIN = 1e-6


def intrinsic_matrix(cam) -> np.ndarray:
    return np.array([[cam["fx"], 0.0, cam["cx"]], [0.0, cam["fy"], cam["cy"]], [0.0, 0.0, 1.0]], dtype=np.float64)


def relative_motion(cam1, cam2):
    """(R, t) with X2 = R X1 + t for camera-space points of frames 1 and 2."""
    T1 = np.asarray(cam1["T_cw"], dtype=np.float64)
    T2 = np.asarray(cam2["T_cw"], dtype=np.float64)
    R = T2[:, :3] @ T1[:, :3].T
    t = T2[:, 3] - R @ T1[:, 3]
    return R, t


def skew(v) -> np.ndarray:
    x, y, z = v
    return np.array([[0.0, -z, y], [z, 0.0, -x], [-y, x, 0.0]])


def fundamental(cam1, cam2) -> np.ndarray:
    """F = K2^-T [t]_x R K1^-1 (maps pixels of frame 1 to lines of frame 2)."""
    R, t = relative_motion(cam1, cam2)
    if np.linalg.norm(t) < T_MIN:
        return np.zeros((3, 3))
    E = skew(t) @ R
    return np.linalg.inv(intrinsic_matrix(cam2)).T @ E @ np.linalg.inv(intrinsic_matrix(cam1))


def epipolar_distance(F, p1, p2) -> np.ndarray:
    """Eq. (18) in float64 for matches p1, p2 given as [2][m] pixel arrays."""
    p1 = np.asarray(p1, dtype=np.float64)
    p2 = np.asarray(p2, dtype=np.float64)
    h1 = np.vstack([p1, np.ones(p1.shape[1])])
    line = F @ h1
    num = np.abs(p2[0] * line[0] + p2[1] * line[1] + line[2])
    with np.errstate(invalid="ignore", divide="ignore"):
        return num / np.sqrt(line[0] ** 2 + line[1] ** 2)


def to_f32_canonical(d) -> np.ndarray:
    """float32 distances with every NaN as the positive quiet NaN."""
    d32 = np.asarray(d, dtype=np.float64).astype(np.float32)
    bits = d32.view(np.uint32).copy()
    bits[np.isnan(d32)] = QNAN_BITS
    return bits.view(np.float32)


def lower_median_f32(x32) -> np.float32:
    """The lower median of float32 values >= 0 (NaN allowed), ordered by bit
    pattern; NaN for an empty set."""
    x32 = np.asarray(x32, dtype=np.float32)
    if x32.size == 0:
        return np.float32(np.nan)
    bits = np.sort(x32.view(np.uint32))
    return bits[(bits.size - 1) // 2:(bits.size - 1) // 2 + 1].view(np.float32)[0]


def verify(cam1, cam2, p1, p2, ids, seg, mp, eps=1.0, tau=0.5, mp_restore=0.0):
    """Eq. (18)-(19) and the restore rule. ids[k] are candidate Gaussians,
    matches seg[k] .. seg[k+1] belong to candidate k. Returns the float32
    distances, d_bar per candidate, the state per candidate and the new MP."""
    F = fundamental(cam1, cam2)
    p1 = np.asarray(p1, dtype=np.float32)
    p2 = np.asarray(p2, dtype=np.float32)
    m = p1.shape[1]
    d32 = to_f32_canonical(epipolar_distance(F, p1, p2))
    ids = np.asarray(ids, dtype=np.int64)
    seg = np.asarray(seg, dtype=np.int64)
    mp_out = np.array(mp, dtype=np.float32, copy=True)
    n = mp_out.size
    K = ids.size
    dbar = np.full(K, np.nan, dtype=np.float32)
    state = np.zeros(K, dtype=np.uint8)
    for k in range(K):
        b, e = seg[k], seg[k + 1]
        if not (0 <= ids[k] < n) or b < 0 or e < b or e > m:
            state[k] = INVALID
            continue
        if e == b:
            state[k] = NO_MATCHES
            continue
        dbar[k] = lower_median_f32(d32[b:e])
        if not mp_out[ids[k]] > np.float32(tau):
            state[k] = NOT_SUPPRESSED
        elif dbar[k] < np.float32(eps):
            state[k] = RESTORED
        else:
            state[k] = KEPT
    # restoring after every decision: a Gaussian listed twice is judged on its
    # MP before any restore
    rest = ids[state == RESTORED]
    mp_out[rest] = np.float32(mp_restore)
    return dict(d=d32, dbar=dbar, state=state, mp=mp_out, F=F)
