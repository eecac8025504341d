"""Pins of the oracle's k < F paths (Sec. 5.3: k contact domains chosen at
random; Sec. 5.6: joints without a contact take random values):

* the finger choice: every eligible finger when k equals their number (so
  k = F keeps contact i on finger i), no set when fewer are eligible, never an
  empty domain, increasing order, and uniform over the k-subsets (chi-square);
* the draws put contact i's point in the domain of its finger and its link on
  that finger (a point of the finger's merged table);
* the random joints of a finger without contact lie within the limits and are
  uniform (chi-square over deciles), independently across fingers;
* realize with k < F: a finger without contact keeps exactly those random
  values, a contact's finger follows its link, and planting an invalid link,
  point or finger order makes the set unrealisable (+inf errors, not valid,
  every finger random) -- the same configuration a set of only unused fingers
  would give.
"""
import dataclasses
import itertools
import math

import numpy as np
import pytest
from scipy.stats import chi2

import oracle
import synth


def _sp(**kw):
    base = dict(draws=400, k=3, mu=0.5, m_edges=8, eps=1e-3, seed=1234)
    base.update(kw)
    return synth.SearchParams(**base)


def test_all_eligible_fingers_when_k_equals_their_number():
    F = 5
    cnt = np.array([[3, 1, 7, 2, 9], [0, 4, 0, 5, 6], [1, 0, 0, 0, 0]], np.uint32)
    out = oracle.choose_fingers(cnt, 5, _sp(k=5), draws=16)
    assert (out[0] == np.arange(F)).all()
    assert (out[1:] == -1).all()                        # fewer than k eligible
    out = oracle.choose_fingers(cnt, 3, _sp(k=3), draws=16)
    assert (out[1] == np.array([1, 3, 4])).all()        # exactly the eligible fingers
    assert (out[2] == -1).all()
    out = oracle.choose_fingers(cnt, 1, _sp(k=1), draws=16)
    assert (out[2] == 0).all()


def test_choice_is_uniform_over_subsets():
    F, k, D = 5, 3, 4000
    cnt = np.ones((3, F), np.uint32)
    out = oracle.choose_fingers(cnt, k, _sp(k=k), draws=D).reshape(-1, k)
    assert (np.diff(out, axis=1) > 0).all()             # increasing finger order
    subsets = {s: i for i, s in enumerate(itertools.combinations(range(F), k))}
    c = np.bincount([subsets[tuple(r)] for r in out], minlength=len(subsets))
    e = len(out) / len(subsets)
    assert ((c - e) ** 2 / e).sum() < chi2.ppf(0.999, len(subsets) - 1)


def test_choice_never_takes_an_empty_domain():
    rng = np.random.default_rng(3)
    cnt = (rng.random((64, 6)) < 0.6).astype(np.uint32) * 5
    out = oracle.choose_fingers(cnt, 2, _sp(k=2), draws=32)
    for g in range(64):
        elig = np.flatnonzero(cnt[g])
        if len(elig) < 2:
            assert (out[g] == -1).all()
        else:
            assert np.isin(out[g], elig).all()
    # a different request id gives different choices
    other = oracle.choose_fingers(cnt, 2, _sp(k=2, request_id=7), draws=32)
    assert (other != out).any()


def test_unused_joints_are_uniform_within_limits():
    w = synth.workload("c3", n_poses=1, with_sdf=False)
    H = w.hand
    sp = _sp(k=3)
    n = 3000
    for f in range(H.n_fingers):
        j = np.flatnonzero(H.joint_finger == f)
        lo, hi = H.limits[j, 0].astype(np.float64), H.limits[j, 1].astype(np.float64)
        u = np.array([(oracle.unused_joints(H, f, sp, g, 0) - lo) / (hi - lo) for g in range(n)])
        assert (u >= 0).all() and (u < 1).all()
        for t in range(len(j)):
            c = np.bincount(np.minimum((u[:, t] * 10).astype(int), 9), minlength=10)
            assert ((c - n / 10) ** 2 / (n / 10)).sum() < chi2.ppf(0.999, 9)
        if len(j) > 1:
            assert abs(np.corrcoef(u[:, 0], u[:, 1])[0, 1]) < 5 / math.sqrt(n)
    # fingers draw from different counters
    a = oracle.unused_joints(H, 0, sp, 5, 1)
    b = oracle.unused_joints(H, 1, sp, 5, 1)
    assert not np.allclose(a[:min(len(a), len(b))], b[:min(len(a), len(b))])


@pytest.fixture(scope="module")
def c3k():
    w = synth.workload("c3", samples=4096, n_poses=64, with_sdf=True)
    sp = dataclasses.replace(w.search, k=3, draws=64)
    fld = oracle.build_field(w.hand, w.field, witness=True, flags=False)
    Q = oracle.query(w.hand, w.field, fld["bits"], w.obj.pts, w.obj.nrm, w.poses, flags=False)
    spt, sln = oracle.draw(w.hand, w.field, fld["bits"], w.obj.pts, w.obj.nrm, w.poses, Q["dom_bits"],
                           Q["dom_count"], sp)
    return w, sp, fld, Q, spt, sln


def test_draws_follow_the_chosen_fingers(c3k):
    w, sp, fld, Q, spt, sln = c3k
    H = w.hand
    fing = oracle.choose_fingers(Q["dom_count"], sp.k, sp)
    P, D, k = spt.shape
    N = w.obj.n
    bits = np.unpackbits(Q["dom_bits"].view(np.uint8), axis=-1, bitorder="little")[..., :N]
    drawn = (fing >= 0).all(-1)
    assert drawn.sum() > 0 and (spt[~drawn] == -1).all()
    used = set()
    for g, d in zip(*np.nonzero(drawn)):
        for i in range(k):
            f = fing[g, d, i]
            used.add(int(f))
            assert bits[g, f, spt[g, d, i]]                 # the point is in its finger's domain
            l = sln[g, d, i]
            assert l >= 0 and H.joint_finger[l] == f        # the link is on that finger
    assert len(used) == H.n_fingers                          # every finger takes part somewhere


def test_realize_k_below_f(c3k):
    w, sp, fld, Q, spt, sln = c3k
    H = w.hand
    V = oracle.verdicts(w.obj.pts, w.obj.nrm, spt, sp)
    acc = oracle.compact(V["verdict"])[:200]
    assert len(acc) > 5
    k = sp.k
    R = oracle.realize(H, w.field, fld["wit"], w.sdf, w.obj.pts, w.obj.nrm, w.poses, spt.reshape(-1, k),
                       sln.reshape(-1, k), sp, acc, w.ik)
    for a, sid in enumerate(acc):
        g, d = divmod(int(sid), sp.draws)
        fingers = H.joint_finger[sln.reshape(-1, k)[sid]]
        for f in range(H.n_fingers):
            j = np.flatnonzero(H.joint_finger == f)
            if f in fingers:
                # the contact's finger: IK from the witness, one ik_finger call
                i = int(np.flatnonzero(fingers == f)[0])
                assert np.isfinite(R["contact_err"][a, i])
            else:
                np.testing.assert_array_equal(R["q"][a, j], oracle.unused_joints(H, f, sp, g, d))
                np.testing.assert_array_equal(R["q0"][a, j], R["q"][a, j])
        # depth over every link of the hand, the unused fingers' included
        assert R["depth"][a] == pytest.approx(oracle.penetration(H, R["q"][a], w.sdf, w.poses[g]), abs=1e-12)


def test_unrealisable_sets(c3k):
    w, sp, fld, Q, spt, sln = c3k
    H = w.hand
    k = sp.k
    V = oracle.verdicts(w.obj.pts, w.obj.nrm, spt, sp)
    acc = oracle.compact(V["verdict"])[:4]
    assert len(acc) == 4
    S, L = spt.reshape(-1, k).copy(), sln.reshape(-1, k).copy()
    L[acc[0], 1] = -1                                  # no hand link at the point
    S[acc[1], 0] = w.obj.n                             # not an object point
    L[acc[2]] = L[acc[2]][::-1]                        # fingers out of order
    R = oracle.realize(H, w.field, fld["wit"], w.sdf, w.obj.pts, w.obj.nrm, w.poses, S, L, sp, acc, w.ik)
    for a in range(3):
        assert np.isinf(R["contact_err"][a]).all() and np.isinf(R["contact_ang"][a]).all()
        assert R["valid"][a] == 0
        g, d = divmod(int(acc[a]), sp.draws)
        for f in range(H.n_fingers):
            j = np.flatnonzero(H.joint_finger == f)
            np.testing.assert_array_equal(R["q"][a, j], oracle.unused_joints(H, f, sp, g, d))
    assert np.isfinite(R["contact_err"][3]).all()     # the untouched set is realised
    with pytest.raises(ValueError):
        oracle.realize(H, w.field, fld["wit"], w.sdf, w.obj.pts, w.obj.nrm, w.poses, S, L, sp,
                       np.array([len(w.poses) * sp.draws], np.int32), w.ik)


def test_link_flags_cover_every_band_decision():
    """The reverse lookup's band flag (Sec. 5.5 link pick): moving each pose
    by 8e-7 m along an axis, or turning it by 8e-7 rad about one, never
    changes a link the oracle does not flag (the bands are 1e-6 m and
    1e-6 rad); on poses moved to put a contact 3e-7 m from a voxel face, the
    links that do change across it are all flagged, and some do."""
    w = synth.workload("c1", n_poses=96)
    ref = oracle.build_field(w.hand, w.field, flags=False)
    Q = oracle.query(w.hand, w.field, ref["bits"], w.obj.pts, w.obj.nrm, w.poses, flags=False)
    spt, sln, lf = oracle.draw(w.hand, w.field, ref["bits"], w.obj.pts, w.obj.nrm, w.poses, Q["dom_bits"],
                               Q["dom_count"], w.search, link_flags=True)
    # relink on the same points gives the same links and flags
    s2, f2 = oracle.relink(w.hand, w.field, ref["bits"], w.obj.pts, w.obj.nrm, w.poses, spt, w.search,
                           dom_count=Q["dom_count"], link_flags=True)
    assert np.array_equal(s2, sln) and np.array_equal(f2, lf)
    on = spt >= 0
    P0 = w.poses.astype(np.float64).reshape(-1, 3, 4)
    for axis in range(3):
        for sgn in (-1.0, 1.0):
            for kind in ("move", "turn"):
                P = P0.copy()
                if kind == "move":
                    P[:, axis, 3] += sgn * 8e-7
                else:
                    a = sgn * 8e-7
                    c, s = math.cos(a), math.sin(a)
                    i, j = [(1, 2), (2, 0), (0, 1)][axis]
                    Rt = np.eye(3)
                    Rt[i, i], Rt[i, j], Rt[j, i], Rt[j, j] = c, -s, s, c
                    P[:, :, :3] = Rt @ P[:, :, :3]
                ln = oracle.relink(w.hand, w.field, ref["bits"], w.obj.pts, w.obj.nrm,
                                   P.reshape(-1, 12).astype(np.float32), spt, w.search, dom_count=Q["dom_count"])
                ch = on & (ln != sln)
                assert (ch & (lf == 0)).sum() == 0, (axis, sgn, kind)
    assert lf[on].mean() < 0.02
    # poses moved so that a contact's point lies 3e-7 m from a voxel face of
    # its finger's window (the synthetic windows have the hand frame's axes):
    # the link must be flagged wherever the other side gives another link
    h = float(np.float32(w.field.h))
    D, k = w.search.draws, w.search.k
    rng = np.random.default_rng(5)
    cand = np.argwhere(on.reshape(-1, k))
    differ = 0
    for s_, i in cand[rng.choice(len(cand), size=240, replace=False)]:
        g = s_ // D
        f = int(w.hand.joint_finger[sln.reshape(-1, k)[s_, i]])
        o = w.field.grid_frame[f].reshape(3, 4)[:, 3].astype(np.float64)
        x = P0[g, :, :3] @ w.obj.pts[spt.reshape(-1, k)[s_, i]].astype(np.float64) + P0[g, :, 3]
        a = int(rng.integers(3))
        u = (x[a] - o[a]) / h
        Pg = P0[g:g + 1].copy()
        Pg[0, a, 3] += (np.round(u) - u) * h + 3e-7
        sp1 = dataclasses.replace(w.search, pose_offset=g)
        one = spt[g:g + 1]
        base, fl = oracle.relink(w.hand, w.field, ref["bits"], w.obj.pts, w.obj.nrm,
                                 Pg.reshape(-1, 12).astype(np.float32), one, sp1,
                                 dom_count=Q["dom_count"][g:g + 1], link_flags=True)
        for sgn in (-1.0, 1.0):
            Pm = Pg.copy()
            Pm[0, a, 3] += sgn * 8e-7
            ln = oracle.relink(w.hand, w.field, ref["bits"], w.obj.pts, w.obj.nrm,
                               Pm.reshape(-1, 12).astype(np.float32), one, sp1, dom_count=Q["dom_count"][g:g + 1])
            ch = (one >= 0) & (ln != base)
            assert (ch & (fl == 0)).sum() == 0, (s_, i, a, sgn)
            differ += int(ch.sum())
    assert differ > 0
