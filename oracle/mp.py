"""FP64 reference of the per-Gaussian motion-probability (MP) update.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Follows Sec. IV-A (Eq. (1)-(13)) and Sec. IV-B (Eq. (17)) step by step, with
the paper's geometric cue (feature reprojection error, Eq. (3)) replaced by a
dense per-pixel depth (+ optional photometric) residual, and the feature set
replaced by the valid pixels around each projected mean at one scale. Readings
of points the paper leaves open are the parameters below; each is listed with
its reason in the design notes of the repository.

Pinned by tests/test_oracle_mp.py: the paper's named special cases (instant
MP: alpha = 1; fixed rate: alpha_min = alpha_max; MP_geo only: K = 1; MP_ins
only: K = 0; stale prior: alpha' = rho alpha), closed forms (entropy of 0.5 is
ln 2; constant observations give zero variance and M_hat = M_p; uniform residual
gives sigma_e = 0), medians against numpy's sort, and a pure-Python brute force
of the whole update on tiny inputs.
"""

from __future__ import annotations

import numpy as np

DEFAULTS = dict(
    lambda_e=2.0,       # Eq. (4): e_ub = mu_e + lambda sigma_e
    sigma_small=1e-3,   # Eq. (5) note: "when sigma_e is small" use the region mean
    e_floor=0.0,        # floor on e_ub (0 = literal)
    sigma_g=0.05,       # Eq. (7): Gamma_geo = exp(-sigma_e,k / sigma_g)
    sigma_c=0.05,       # Eq. (11): C = exp(-sigma_e,G / sigma_c)
    lambda_u=1.0,       # Eq. (10)
    eps=1e-6,           # Eq. (10)
    alpha_min=0.1,      # Eq. (11)
    alpha_max=0.8,
    rho=0.5,            # Eq. (17)
    radius_px=2.0,      # Eq. (1): association radius r_s at one scale
    sigma_w=1.0,        # soft association kernel width
    beta_color=0.0,     # photometric share of the residual cue
    prune_above=2.0,    # prune flag M > prune_above (disabled when >= 1)
    logodds_eps=0.01,
    logodds_max=float(np.log(99.0)),
    mode=0,             # 0: exponential smoothing Eq. (9); 1: log-odds variant
    u_norm=0,           # 0: min-max within the frame; 1: divide by ln2 + lambda_u/4
)


def lower_median(v):
    v = np.sort(np.asarray(v, np.float64))
    if v.size == 0:
        return None
    return float(v[(v.size - 1) // 2])


def residual(depth, target_depth, color=None, target_color=None, beta=0.0):
    e = np.abs(np.asarray(depth, np.float64) - np.asarray(target_depth, np.float64))
    if beta != 0.0:
        e = e + beta * np.abs(np.asarray(color, np.float64) - np.asarray(target_color, np.float64)).sum(axis=0)
    return e


def region_stats(e, valid, inst, n_inst):
    """Eq. (4): mean and population std of e over the valid pixels of each
    region k = 0 (background) .. K. Regions with no valid pixel get 0, 0."""
    mu = np.zeros(n_inst + 1)
    sd = np.zeros(n_inst + 1)
    cnt = np.zeros(n_inst + 1, np.int64)
    for k in range(n_inst + 1):
        sel = valid & (inst == k)
        cnt[k] = sel.sum()
        if cnt[k] > 0:
            mu[k] = e[sel].mean()
            sd[k] = np.sqrt(((e[sel] - mu[k]) ** 2).mean())
    return mu, sd, cnt


def pixel_mp(e, valid, inst, prior, conf, p):
    """Eq. (2), (4)-(7): per-pixel fused MP M_p and the pieces it is made of."""
    K = len(prior) - 1
    mu, sd, cnt = region_stats(e, valid, inst, K)
    e_ub = np.maximum(mu + p["lambda_e"] * sd, p["e_floor"])
    k = inst
    e_t = np.where(sd[k] < p["sigma_small"], mu[k], e)
    ub = e_ub[k]
    mp_geo = np.where(ub > 0, np.clip(e_t / np.where(ub > 0, ub, 1.0), 0.0, 1.0), 0.0)
    mp_ins = np.asarray(prior, np.float64)[k]
    g_ins = np.asarray(conf, np.float64)[k]
    g_geo = np.exp(-sd[k] / p["sigma_g"])
    den = g_ins + g_geo
    gain = np.where(den > 0, g_geo / np.where(den > 0, den, 1.0), 0.5)
    Mp = (1.0 - gain) * mp_ins + gain * mp_geo
    return dict(M_p=Mp, mp_geo=mp_geo, mp_ins=mp_ins, gain=gain, mu=mu, sd=sd, cnt=cnt, e_ub=e_ub)


def window_aggregate(mean2d_f32, kept, width, height, valid, radius_px, sigma_w, Mp, e):
    """Eq. (1) and (8) at one scale, for every visible Gaussian at once.

    N(G) = valid pixels whose centre lies within radius_px of the projected
    mean; membership is decided in float32 without fused multiply-add
    (dx = i - u_x rounded, then dx*dx + dy*dy rounded), the precision the GPU
    kernel decides it in. Returns per Gaussian: |N(G)|, the kernel-weighted
    mean of M_p (weights exp(-d^2 / (2 sigma_w^2)) with float64 distances),
    the population variance of M_p and the population std of e over N(G)."""
    u = np.asarray(mean2d_f32, np.float32)
    N = u.shape[1]
    r = np.float32(radius_px)
    r2 = np.float32(r * r)
    vis = np.asarray(kept, bool) & (u[0] >= 0) & (u[0] <= width - 1) & (u[1] >= 0) & (u[1] <= height - 1)
    rr = int(np.ceil(radius_px)) + 1
    cx = np.floor(u[0]).astype(np.int64)
    cy = np.floor(u[1]).astype(np.int64)
    offs = [(ox, oy) for oy in range(-rr, rr + 1) for ox in range(-rr, rr + 1)]
    X = np.stack([cx + ox for ox, oy in offs], axis=1)          # [N, S]
    Y = np.stack([cy + oy for ox, oy in offs], axis=1)
    inside = (X >= 0) & (X <= width - 1) & (Y >= 0) & (Y <= height - 1)
    Xc = np.clip(X, 0, width - 1)
    Yc = np.clip(Y, 0, height - 1)
    idx = Yc * width + Xc
    dx = (Xc.astype(np.float32) - u[0][:, None]).astype(np.float32)
    dy = (Yc.astype(np.float32) - u[1][:, None]).astype(np.float32)
    d2 = ((dx * dx).astype(np.float32) + (dy * dy).astype(np.float32)).astype(np.float32)
    member = inside & (d2 <= r2) & valid[idx] & vis[:, None]
    n = member.sum(axis=1)
    d2_64 = (Xc - u[0][:, None].astype(np.float64)) ** 2 + (Yc - u[1][:, None].astype(np.float64)) ** 2
    w = np.where(member, np.exp(-d2_64 / (2.0 * sigma_w ** 2)), 0.0)
    m = np.where(member, Mp[idx], 0.0)
    ev = np.where(member, e[idx], 0.0)
    nn = np.maximum(n, 1)
    sw = w.sum(axis=1)
    M_hat = np.where(n > 0, (w * m).sum(axis=1) / np.where(sw > 0, sw, 1.0), 0.0)
    mm = m.sum(axis=1) / nn
    var = np.where(member, (m - mm[:, None]) ** 2, 0.0).sum(axis=1) / nn
    me = ev.sum(axis=1) / nn
    sd_e = np.sqrt(np.where(member, (ev - me[:, None]) ** 2, 0.0).sum(axis=1) / nn)
    return n, M_hat, var, sd_e


def mp_update(inp: dict, params: dict | None = None, seg_updated: bool = True, mlp_mp=None) -> dict:
    """One frame of the MP update. `inp` holds width, height, depth[P],
    target_depth[P] (0 = invalid), color/target_color [3,P] (used when
    beta_color > 0), instance_id[P], inst_prior[K+1], inst_conf[K+1],
    mean2d[2,N] (float32), culled[N], mp[N] (state M^{t-1})."""
    p = dict(DEFAULTS)
    if params:
        p.update(params)
    W, H = inp["width"], inp["height"]
    D = np.asarray(inp["depth"], np.float64)
    Dg = np.asarray(inp["target_depth"], np.float64)
    valid = Dg > 0
    e = residual(D, Dg, inp.get("color"), inp.get("target_color"), p["beta_color"])
    inst = np.asarray(inp["instance_id"], np.int64)
    pm = pixel_mp(e, valid, inst, inp["inst_prior"], inp["inst_conf"], p)
    Mp = pm["M_p"] if mlp_mp is None else np.asarray(mlp_mp, np.float64)

    mprev = np.asarray(inp["mp"], np.float64)
    N = mprev.shape[0]
    kept = ~np.asarray(inp["culled"], bool)
    nobs, M_hat, var, sd_e = window_aggregate(inp["mean2d"], kept, W, H, valid, p["radius_px"], p["sigma_w"],
                                              Mp, e)                # Eq. (1), (8)
    observed = nobs > 0

    eps = p["eps"]
    Mq = mprev
    U = -Mq * np.log(Mq + eps) - (1 - Mq) * np.log(1 - Mq + eps) + p["lambda_u"] * var  # Eq. (10)
    Ut = np.zeros(N)
    if observed.any():
        if p["u_norm"] == 0:
            umin, umax = U[observed].min(), U[observed].max()
            if umax > umin:
                Ut[observed] = (U[observed] - umin) / (umax - umin)
        else:
            Ut[observed] = np.clip(U[observed] / (np.log(2.0) + p["lambda_u"] / 4.0), 0.0, 1.0)
    Cg = np.exp(-sd_e / p["sigma_c"])
    amin, amax = p["alpha_min"], p["alpha_max"]
    alpha = np.clip(amin + (amax - amin) * (1.0 - Ut) * Cg, amin, amax)  # Eq. (11)
    alpha_p = alpha if seg_updated else p["rho"] * alpha                  # Eq. (17)
    alpha_p = np.where(observed, alpha_p, 0.0)
    Ut = np.where(observed, Ut, 0.0)

    new = mprev.copy()
    if p["mode"] == 0:
        upd = (1 - alpha_p) * mprev + alpha_p * M_hat                        # Eq. (9)
    else:
        le = p["logodds_eps"]
        lo = lambda x: np.log(x / (1 - x))
        l0 = lo(np.clip(mprev, le, 1 - le))
        l1 = np.clip(l0 + alpha_p * lo(np.clip(M_hat, le, 1 - le)), -p["logodds_max"], p["logodds_max"])
        upd = 1.0 / (1.0 + np.exp(-l1))
    new[observed] = upd[observed]

    med = lower_median(new[observed]) if observed.any() else None
    tau = max(med, 0.5) if med is not None else 0.5                       # Eq. (12)
    dynamic = new > tau
    ubar = lower_median(Ut[observed]) if observed.any() else 0.0          # Eq. (13)
    prune = new > p["prune_above"]
    stats = dict(U_bar=ubar, tau=tau, n_obs=int(observed.sum()), n_dyn=int(dynamic.sum()),
                 n_prune=int(prune.sum()), median=med if med is not None else 0.0)
    return dict(mp=new, M_hat=M_hat, var=var, sd_e=sd_e, nobs=nobs, observed=observed, U=U, U_tilde=Ut,
                alpha=alpha_p, dynamic=dynamic, prune=prune, stats=stats, e=e, **pm, M_p_used=Mp)
