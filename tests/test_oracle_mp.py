"""Pins of the FP64 MP-update oracle (CPU only): the special cases the paper
names (Table VII / VIII variants, Eq. (17)), closed forms, and a pure-Python
brute force of Eq. (1)-(13) on tiny inputs."""

import math

import numpy as np

from paper_2602_21644_amd import synth


def small_inputs(seed=1, n=400, w=40, h=30, k=3):
    return synth.mp_frame_inputs(seed, n, w, h, n_inst=k)


def test_instant_mp_alpha_one(orc):
    """alpha_min = alpha_max = 1: 'Instant MP', M^t = M_hat (Sec. V-C)."""
    inp = small_inputs()
    r = orc.mp.mp_update(inp, dict(alpha_min=1.0, alpha_max=1.0))
    obs = r["observed"]
    assert obs.sum() > 100
    np.testing.assert_allclose(r["mp"][obs], r["M_hat"][obs], atol=1e-15)
    np.testing.assert_array_equal(r["mp"][~obs], inp["mp"][~obs].astype(np.float64))


def test_fixed_rate(orc):
    """alpha_min = alpha_max = a: fixed exponential smoothing, Eq. (9)."""
    inp = small_inputs(2)
    r = orc.mp.mp_update(inp, dict(alpha_min=0.3, alpha_max=0.3))
    obs = r["observed"]
    m0 = inp["mp"].astype(np.float64)
    np.testing.assert_allclose(r["mp"][obs], 0.7 * m0[obs] + 0.3 * r["M_hat"][obs], atol=1e-15)


def test_stale_prior_rho(orc):
    """Eq. (17): without a prior refresh the rate is rho * alpha."""
    inp = small_inputs(3)
    a = orc.mp.mp_update(inp, seg_updated=True)
    b = orc.mp.mp_update(inp, seg_updated=False)
    np.testing.assert_allclose(b["alpha"], 0.5 * a["alpha"], atol=1e-15)


def test_fusion_extremes(orc):
    """c_bg = c_k = 0 gives K = 1 (MP_geo only); sigma_g -> 0+ gives K = 0
    (MP_ins only) wherever the region has sigma_e > 0 (Table VIII variants)."""
    inp = small_inputs(4)
    i1 = dict(inp)
    i1["inst_conf"] = np.zeros_like(inp["inst_conf"])
    r = orc.mp.mp_update(i1)
    np.testing.assert_allclose(r["M_p"], r["mp_geo"], atol=1e-15)
    r = orc.mp.mp_update(inp, dict(sigma_g=1e-300))
    sd = r["sd"][inp["instance_id"]]
    sel = sd > 0
    np.testing.assert_allclose(r["M_p"][sel], r["mp_ins"][sel], atol=1e-15)


def test_entropy_half_is_ln2(orc):
    """Eq. (10) with M^{t-1} = 0.5 and lambda_u = 0: U -> ln 2 as eps -> 0."""
    inp = small_inputs(5)
    inp["mp"] = np.full_like(inp["mp"], 0.5)
    r = orc.mp.mp_update(inp, dict(lambda_u=0.0, eps=1e-14))
    np.testing.assert_allclose(r["U"], math.log(2.0), rtol=1e-12)


def test_constant_observation_and_uniform_residual(orc):
    """A uniform residual e = e0 gives sigma_e = 0 in every region, hence
    MP_geo = min(1, e0 / max(e0, e_floor)), Gamma_geo = 1, a constant M_p per
    region, zero window variance and M_hat = M_p inside one region."""
    inp = small_inputs(6)
    inp["target_depth"] = np.where(inp["target_depth"] > 0, inp["depth"] + np.float32(0.02), 0).astype(np.float32)
    inp["depth"] = inp["depth"].astype(np.float32)
    e0 = np.abs(inp["depth"].astype(np.float64) - inp["target_depth"].astype(np.float64))
    inp["target_depth"] = np.where(inp["target_depth"] > 0, inp["depth"].astype(np.float64) + 0.02, 0)
    inp["depth"] = inp["depth"].astype(np.float64)
    for floor, expect in ((0.0, 1.0), (0.08, 0.25)):
        r = orc.mp.mp_update(inp, dict(e_floor=floor))
        assert np.all(r["sd"] < 1e-12)
        valid = inp["target_depth"] > 0
        np.testing.assert_allclose(r["mp_geo"][valid], expect, rtol=1e-9)
    r = orc.mp.mp_update(inp)
    inst = inp["instance_id"]
    for k in np.nonzero(r["observed"])[0][:50]:
        # neighbourhood pixels all from region 0 -> constant M_p
        u = inp["mean2d"][:, k]
        i0, j0 = int(np.floor(u[0])), int(np.floor(u[1]))
        xs = np.clip(np.arange(i0 - 3, i0 + 4), 0, inp["width"] - 1)
        ys = np.clip(np.arange(j0 - 3, j0 + 4), 0, inp["height"] - 1)
        if np.all(inst.reshape(inp["height"], inp["width"])[np.ix_(ys, xs)] == 0):
            assert r["var"][k] < 1e-24
            np.testing.assert_allclose(r["M_hat"][k], r["M_p"][inst == 0][0], rtol=1e-12)


def test_medians(orc):
    v = np.random.default_rng(0).random(101)
    assert orc.mp.lower_median(v) == np.median(v)
    v = np.random.default_rng(1).random(100)
    assert orc.mp.lower_median(v) == np.sort(v)[49]


def _brute_update(inp, p, seg_updated=True):
    """Pure-Python loops over pixels and Gaussians (tiny inputs only)."""
    W, H = inp["width"], inp["height"]
    P = W * H
    K = len(inp["inst_prior"]) - 1
    D = [float(x) for x in inp["depth"]]
    Dg = [float(x) for x in inp["target_depth"]]
    ins = [int(x) for x in inp["instance_id"]]
    e = [abs(D[i] - Dg[i]) for i in range(P)]
    stats = []
    for k in range(K + 1):
        vals = [e[i] for i in range(P) if ins[i] == k and Dg[i] > 0]
        if vals:
            m = sum(vals) / len(vals)
            s = math.sqrt(sum((v - m) ** 2 for v in vals) / len(vals))
        else:
            m = s = 0.0
        stats.append((m, s))
    Mp = []
    for i in range(P):
        m, s = stats[ins[i]]
        ub = max(m + p["lambda_e"] * s, p["e_floor"])
        et = m if s < p["sigma_small"] else e[i]
        geo = min(max(et / ub, 0.0), 1.0) if ub > 0 else 0.0
        gi = float(inp["inst_conf"][ins[i]])
        gg = math.exp(-s / p["sigma_g"])
        Kp = gg / (gi + gg) if gi + gg > 0 else 0.5
        Mp.append((1 - Kp) * float(inp["inst_prior"][ins[i]]) + Kp * geo)
    N = len(inp["mp"])
    res = []
    for k in range(N):
        ux, uy = np.float32(inp["mean2d"][0, k]), np.float32(inp["mean2d"][1, k])
        if inp["culled"][k] or not (0 <= ux <= W - 1 and 0 <= uy <= H - 1):
            res.append(None)
            continue
        ws, ms, es = [], [], []
        for j in range(H):
            for i in range(W):
                dx = np.float32(np.float32(i) - ux)
                dy = np.float32(np.float32(j) - uy)
                d2 = np.float32(np.float32(dx * dx) + np.float32(dy * dy))
                if d2 <= np.float32(p["radius_px"] ** 2) and Dg[j * W + i] > 0:
                    dd = (i - float(ux)) ** 2 + (j - float(uy)) ** 2
                    ws.append(math.exp(-dd / (2 * p["sigma_w"] ** 2)))
                    ms.append(Mp[j * W + i])
                    es.append(e[j * W + i])
        if not ws:
            res.append(None)
            continue
        mh = sum(a * b for a, b in zip(ws, ms)) / sum(ws)
        mm = sum(ms) / len(ms)
        var = sum((x - mm) ** 2 for x in ms) / len(ms)
        em = sum(es) / len(es)
        sde = math.sqrt(sum((x - em) ** 2 for x in es) / len(es))
        M0 = float(inp["mp"][k])
        U = -M0 * math.log(M0 + p["eps"]) - (1 - M0) * math.log(1 - M0 + p["eps"]) + p["lambda_u"] * var
        res.append((mh, var, sde, U))
    Us = [r[3] for r in res if r is not None]
    umin, umax = min(Us), max(Us)
    out = []
    for k in range(N):
        if res[k] is None:
            out.append(float(inp["mp"][k]))
            continue
        mh, var, sde, U = res[k]
        Ut = (U - umin) / (umax - umin) if umax > umin else 0.0
        a = p["alpha_min"] + (p["alpha_max"] - p["alpha_min"]) * (1 - Ut) * math.exp(-sde / p["sigma_c"])
        a = min(max(a, p["alpha_min"]), p["alpha_max"])
        if not seg_updated:
            a *= p["rho"]
        out.append((1 - a) * float(inp["mp"][k]) + a * mh)
    return out


def test_bruteforce_tiny(orc):
    inp = synth.mp_frame_inputs(11, 30, 8, 6, n_inst=1)
    assert (~inp["culled"]).sum() > 10
    p = dict(orc.mp.DEFAULTS)
    for seg in (True, False):
        r = orc.mp.mp_update(inp, seg_updated=seg)
        ref = _brute_update(inp, p, seg)
        np.testing.assert_allclose(r["mp"], ref, rtol=1e-12, atol=1e-14)
