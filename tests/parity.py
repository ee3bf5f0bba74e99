"""Parity between the GPU renders and the FP64 oracle.

The gate (per the tolerance the method is held to):
  * a path is a *tie* when its ray-tree signature differs from the oracle's: the
    closest-hit id at any depth, or a shadow state whose oracle contribution
    exceeds 1e-4;
  * ties may be at most 1e-4 of the paths (at least one is allowed on a small
    sample), and every tie must be *certified*: the oracle's margin at the first
    decision where the two disagree is below 1e-3 (an FP32/FP64 rounding flip,
    not a bug);
  * on every other path, every radiance channel agrees to 1e-4 absolute.
"""
from __future__ import annotations

import math

import numpy as np

TIE_BUDGET = 1e-4
RADIANCE_TOL = 1e-4
CERT_MARGIN = 1e-3
CONTRIB_MIN = 1e-4


def gpu_flat(out: dict) -> dict:
    """GPU outputs [2,H,W,...] -> arrays indexed by path id eye*H*W + y*W + x."""
    g = {}
    for k in ("radiance", "hit_t", "hit_prim", "path_prims", "shadow_state"):
        if k in out and out[k] is not None:
            a = out[k].cpu().numpy()
            g[k] = a.reshape((a.shape[0] * a.shape[1] * a.shape[2],) + a.shape[3:])
    return g


def clopper_pearson_upper(k: int, n: int, conf: float = 0.95) -> float:
    from scipy.stats import beta
    if k >= n:
        return 1.0
    return float(beta.ppf(conf, k + 1, n - k))


def compare(g: dict, orc: dict, samples=None, tol=RADIANCE_TOL, allow_min_one=True) -> dict:
    """Compare GPU flat outputs with an oracle result on the oracle's sample of paths."""
    idx = orc["samples"] if samples is None else np.asarray(samples)
    n = len(idx)
    rad = g["radiance"][idx].astype(np.float64)
    pp = g["path_prims"][idx]
    ss = g["shadow_state"][idx]
    opp, oss = orc["path_prims"], orc["shadow_state"]
    contrib = orc["shadow_contrib"]
    prim_diff = pp != opp                                    # [n, D+1]
    shadow_diff = (ss != oss) & (contrib > CONTRIB_MIN)      # [n, D+1, L]
    tie = prim_diff.any(axis=1) | shadow_diff.reshape(n, -1).any(axis=1)
    err = np.abs(rad - orc["radiance"]).max(axis=1)
    nontie = ~tie
    uncertified = []
    D1 = opp.shape[1]
    for k in np.nonzero(tie)[0]:
        margin = None
        for d in range(D1):
            if shadow_diff[k, d].any() and not prim_diff[k, :d + 1].any():
                ls = np.nonzero(shadow_diff[k, d])[0]
                margin = float(orc["shadow_margin"][k, d, ls].min())
                break
            if prim_diff[k, d]:
                margin = float(orc["hit_margin"][k, d])
                break
        if margin is None or not margin < CERT_MARGIN:
            uncertified.append((int(idx[k]), margin))
    n_tie = int(tie.sum())
    budget = TIE_BUDGET * n
    if allow_min_one:
        budget = max(budget, 1.0)
    res = {
        "n": n, "ties": n_tie, "tie_rate": n_tie / max(n, 1), "tie_budget": budget,
        "tie_rate_upper95": clopper_pearson_upper(n_tie, n) if n else 1.0,
        "uncertified": uncertified, "max_err": float(err[nontie].max()) if nontie.any() else 0.0,
        "worst": int(idx[nontie][np.argmax(err[nontie])]) if nontie.any() else -1,
        "tie_ids": [int(x) for x in idx[tie][:20]],
    }
    # primary hit distance on agreeing paths (diagnostic)
    ok = nontie & (orc["hit_prim"] >= 0)
    if ok.any():
        t_g = g["hit_t"][idx][ok].astype(np.float64)
        t_o = orc["hit_t"][ok]
        res["max_rel_t_err"] = float((np.abs(t_g - t_o) / np.maximum(1.0, t_o)).max())
    res["passed"] = bool(n_tie <= budget and not uncertified and res["max_err"] <= tol)
    return res


def assert_parity(res: dict, tol=RADIANCE_TOL):
    msg = (f"n={res['n']} ties={res['ties']} (budget {res['tie_budget']:.2f}) uncertified={res['uncertified'][:5]} "
           f"max_err={res['max_err']:.3g} (worst path {res['worst']}) ties at {res['tie_ids'][:8]}")
    assert res["ties"] <= res["tie_budget"], msg
    assert not res["uncertified"], msg
    assert res["max_err"] <= tol, msg
    if "max_rel_t_err" in res:
        assert res["max_rel_t_err"] <= 1e-5, msg + f" t_err={res['max_rel_t_err']:.3g}"
