"""The realize parity bar (Sec. 5.5 IK + Sec. 3.2 penetration and validity).

On every set the oracle does not flag: the link end points of the final
configuration, the contact errors and the penetration depth agree within
1e-5 m, and validity is identical.  A set is flagged when one of its discrete
choices lies within a rounding band: the reverse lookup's voxel face or bin
boundary, the IK's choice between two distant capsule candidates, or an
acceptance quantity at its threshold.  Flagged sets are counted; their rate is
bounded by what the bands cover (about 2 band/h per coordinate and contact for
the voxel faces, about as much again for the candidate ties).
"""
import numpy as np

import oracle

TOL = 1e-5
MAX_FLAGGED = 0.04


def endpoint_deviation(hand, qa, qb) -> np.ndarray:
    """Per set, the largest coordinate difference of any capsule end point
    between configurations qa and qb (base frame, metres)."""
    out = np.zeros(len(qa))
    caps = [np.asarray(hand.capsule[l], np.float64) for l in range(hand.n_joints)]
    for a in range(len(qa)):
        if np.isnan(qa[a]).any() or np.isnan(qb[a]).any():
            out[a] = 0.0 if (np.isnan(qa[a]) == np.isnan(qb[a])).all() else np.inf
            continue
        Ta, Tb = oracle.fk(hand, qa[a]), oracle.fk(hand, qb[a])
        d = 0.0
        for l, cap in enumerate(caps):
            for e in (cap[:3], cap[3:6]):
                pe = np.append(e, 1.0)
                d = max(d, np.abs(Ta[l].reshape(3, 4) @ pe - Tb[l].reshape(3, 4) @ pe).max())
        out[a] = d
    return out


def _dev(a, b):
    """|a - b| with equal infinities (unrealisable contacts) and equal NaNs counted as 0."""
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    same = (a == b) | (np.isnan(a) & np.isnan(b))
    with np.errstate(invalid="ignore"):
        d = np.abs(a - b)
    return np.where(same, 0.0, np.where(np.isnan(d), np.inf, d))


def check_realize(hand, R, q, err, depth, valid, max_flagged=MAX_FLAGGED) -> dict:
    """Assert the bar on GPU outputs (q [n][J], err [n][k], depth [n], valid [n])
    against the oracle's realize R over the same sets.  Returns the counts."""
    n = len(valid)
    fl = np.asarray(R["rflag"]) != 0
    ep = endpoint_deviation(hand, np.asarray(q, np.float64), R["q"])
    derr = _dev(err, R["contact_err"]).max(axis=1)
    ddep = _dev(depth, R["depth"])
    dval = np.asarray(valid).astype(bool) != np.asarray(R["valid"]).astype(bool)
    bad = (ep > TOL) | (derr > TOL) | (ddep > TOL) | dval
    off = np.flatnonzero(bad & ~fl)
    assert off.size == 0, [
        dict(set=int(a), endpoints=float(ep[a]), err=float(derr[a]), depth=float(ddep[a]), valid=bool(dval[a]))
        for a in off[:8]]
    assert fl.sum() <= max(3, max_flagged * n), (int(fl.sum()), n)
    return {"sets": n, "flagged": int(fl.sum()), "deviating": int(bad.sum()),
            "worst_unflagged": float(max(ep[~fl].max(initial=0), derr[~fl].max(initial=0),
                                         ddep[~fl].max(initial=0)))}
