"""Pins of the oracle's second contact round on the unused fingers (Sec. 5.3
additional search phase; Sec. 5.6, the general form).

What fixes it, independently of the oracle's own code:
- the extended set holds every round-1 contact unchanged, plus k_add contacts
  on fingers the round-1 set does not use, all in increasing finger order;
- each new point lies in its finger's domain (the domain bits), each new link
  is a link of that finger whose table bit is set at the point's voxel and bin
  (voxel from the window frame, bin from a KD-tree over the bin centres);
- the new fingers are uniform over the k_add-subsets of the eligible unused
  fingers (chi-squared), never an empty domain, and a set with too few
  eligible fingers is not extended;
- adding contacts never raises t* (the LP over more wrench columns);
- results are keyed by the global pose and draw index (a subset, or a pose
  run alone at its offset, gives the same sets).
"""
import dataclasses
import itertools

import numpy as np
import pytest
from scipy.spatial import cKDTree
from scipy.stats import chi2

import oracle
import synth


@pytest.fixture(scope="module")
def c3k():
    w = synth.workload("c3", samples=4096, n_poses=96, n_points=4096, with_sdf=False)
    w = dataclasses.replace(w, search=dataclasses.replace(w.search, k=2, draws=32))
    ref = oracle.build_field(w.hand, w.field, flags=False)
    Q = oracle.query(w.hand, w.field, ref["bits"], w.obj.pts, w.obj.nrm, w.poses, flags=False)
    spt, sln = oracle.draw(w.hand, w.field, ref["bits"], w.obj.pts, w.obj.nrm, w.poses, Q["dom_bits"],
                           Q["dom_count"], w.search)
    V = oracle.verdicts(w.obj.pts, w.obj.nrm, spt, w.search)
    return w, ref, Q, spt, sln, V


def _take(spt, sln, V):
    P, D, _ = spt.shape
    return ((spt >= 0).all(-1) & (sln >= 0).all(-1) & (V["verdict"].reshape(P, D) == 0)).astype(np.uint8)


def test_extended_sets_keep_round_one_and_add_unused_fingers(c3k):
    w, ref, Q, spt, sln, V = c3k
    take = _take(spt, sln, V)
    k_add = 2
    e_pt, e_ln, e_fl = oracle.extend(w.hand, w.field, ref["bits"], w.obj.pts, w.obj.nrm, w.poses, Q["dom_bits"],
                                     Q["dom_count"], spt, sln, take, k_add, w.search, request_id=4)
    P, D, k1 = spt.shape
    jf = w.hand.joint_finger
    G, B = w.field.grid, w.field.bins
    h = float(np.float32(w.field.h))
    tree = cKDTree(oracle.bin_centers(B))
    NW = Q["dom_bits"].shape[-1]
    n_ext = checked = 0
    for g, d in zip(*np.nonzero(take)):
        if e_pt[g, d, 0] < 0:
            # not extended: fewer than k_add eligible unused fingers
            used = set(jf[sln[g, d]])
            elig = [f for f in range(w.hand.n_fingers) if f not in used and Q["dom_count"][g, f] > 0]
            assert len(elig) < k_add and (e_pt[g, d] == -1).all()
            continue
        n_ext += 1
        fing = jf[e_ln[g, d]]
        assert (np.diff(fing) > 0).all(), "contacts not in increasing finger order"
        old = {(int(p), int(l)) for p, l in zip(spt[g, d], sln[g, d])}
        new = [(int(p), int(l)) for p, l in zip(e_pt[g, d], e_ln[g, d]) if (int(p), int(l)) not in old]
        assert old <= {(int(p), int(l)) for p, l in zip(e_pt[g, d], e_ln[g, d])}
        assert len(new) == k_add
        P0 = w.poses[g].reshape(3, 4).astype(np.float64)
        for p, l in new:
            f = int(jf[l])
            assert f not in set(jf[sln[g, d]])
            assert (Q["dom_bits"][g, f, p // 32] >> np.uint32(p % 32)) & 1, "new point outside its domain"
            x = P0[:, :3] @ w.obj.pts[p].astype(np.float64) + P0[:, 3]
            n = -(P0[:, :3] @ w.obj.nrm[p].astype(np.float64))
            Fw = w.field.grid_frame[f].reshape(3, 4).astype(np.float64)
            u = Fw[:, :3].T @ (x - Fw[:, 3]) / h
            v = np.floor(u).astype(int)
            b = int(tree.query(n / np.linalg.norm(n))[1])
            near = (np.minimum(u - v, 1 - (u - v)).min() * h < 1e-6)
            if near:
                continue
            vi = (v[2] * G + v[1]) * G + v[0]
            assert (ref["bits"][l, vi, b // 32] >> np.uint32(b % 32)) & 1, "new link not hit at the point"
            checked += 1
    assert n_ext > 500 and checked > 500
    assert NW == (w.obj.n + 31) // 32
    # sets not taken stay -1
    assert (e_pt[take == 0] == -1).all() and (e_ln[take == 0] == -1).all()


def test_adding_contacts_never_raises_tstar(c3k):
    w, ref, Q, spt, sln, V = c3k
    take = _take(spt, sln, V)
    e_pt, e_ln, _ = oracle.extend(w.hand, w.field, ref["bits"], w.obj.pts, w.obj.nrm, w.poses, Q["dom_bits"],
                                  Q["dom_count"], spt, sln, take, 2, w.search, request_id=4)
    sp2 = dataclasses.replace(w.search, k=4)
    V2 = oracle.verdicts(w.obj.pts, w.obj.nrm, e_pt, sp2)
    P, D, _ = spt.shape
    t1 = V["tstar"].reshape(P, D)
    t2 = V2["tstar"].reshape(P, D)
    ext = e_pt[..., 0] >= 0
    assert ext.sum() > 500
    assert (t2[ext] <= t1[ext] + 1e-12).all()
    # some unstable round-1 sets become stable with the added contacts
    assert V2["verdict"].reshape(P, D)[ext].sum() > 0


def test_new_fingers_uniform_over_subsets():
    """All five fingers eligible, one round-1 contact on finger 0: the two new
    fingers are uniform over the 6 pairs of fingers 1..4.  Finger f's domain is
    the single point f, so a new contact's point names its finger."""
    w = synth.workload("c3", samples=1024, n_poses=4000, n_points=64, with_sdf=False)
    F = w.hand.n_fingers
    P, D = 4000, 2
    dom_bits = np.zeros((P, F, 2), np.uint32)
    for f in range(F):
        dom_bits[:, f, 0] = np.uint32(1 << f)
    dom_count = np.ones((P, F), np.uint32)
    first0 = int(w.hand.finger_joints(0)[0])
    spt = np.zeros((P, D, 1), np.int32)
    sln = np.full((P, D, 1), first0, np.int32)
    take = np.ones((P, D), np.uint8)
    bits = np.zeros((w.hand.n_joints, w.field.grid ** 3, w.field.bins // 32), np.uint32)
    e_pt, e_ln, _ = oracle.extend(w.hand, w.field, bits, w.obj.pts, w.obj.nrm, w.poses, dom_bits, dom_count,
                                  spt, sln, take, 2, w.search, request_id=1)
    assert (e_pt[..., 0] == 0).all() and (e_ln[..., 0] == first0).all()
    # no table bit is set: the new contacts have no link (unrealisable), their points are their fingers
    assert (e_ln[..., 1:] == -1).all()
    pairs = [tuple(int(x) for x in fs[1:]) for fs in e_pt.reshape(-1, 3)]
    combos = list(itertools.combinations(range(1, F), 2))
    counts = np.array([pairs.count(c) for c in combos])
    assert counts.sum() == P * D
    exp = P * D / len(combos)
    stat = ((counts - exp) ** 2 / exp).sum()
    assert stat < chi2.ppf(0.999, len(combos) - 1)


def test_too_few_eligible_fingers_and_empty_domains():
    """Finger f's domain is the single point f (or empty), so points name fingers."""
    w = synth.workload("c3", samples=1024, n_poses=64, n_points=64, with_sdf=False)
    F = w.hand.n_fingers
    P, D = 64, 4
    dom_bits = np.zeros((P, F, 2), np.uint32)
    for f in range(F):
        dom_bits[:, f, 0] = np.uint32(1 << f)
    dom_count = np.ones((P, F), np.uint32)
    dom_count[:, 3] = 0                          # finger 3 never eligible
    dom_bits[:, 3] = 0
    dom_count[:32, 4] = 0                        # finger 4 not eligible on half the poses
    dom_bits[:32, 4] = 0
    f0, f1 = int(w.hand.finger_joints(0)[0]), int(w.hand.finger_joints(1)[0])
    spt = np.tile(np.array([0, 1], np.int32), (P, D, 1))
    sln = np.tile(np.array([f0, f1], np.int32), (P, D, 1))
    take = np.ones((P, D), np.uint8)
    bits = np.zeros((w.hand.n_joints, w.field.grid ** 3, w.field.bins // 32), np.uint32)
    e_pt, e_ln, _ = oracle.extend(w.hand, w.field, bits, w.obj.pts, w.obj.nrm, w.poses, dom_bits, dom_count,
                                  spt, sln, take, 2, w.search)
    # poses 0..31: only finger 2 is eligible -> not extended; 32..63: fingers 2 and 4
    assert (e_pt[:32] == -1).all() and (e_ln[:32] == -1).all()
    assert (e_pt[32:] == np.array([0, 1, 2, 4])).all()
    assert (e_ln[32:, :, :2] == np.array([f0, f1])).all()
    # k_add = 1 on poses 0..31 adds finger 2
    e_pt, e_ln, _ = oracle.extend(w.hand, w.field, bits, w.obj.pts, w.obj.nrm, w.poses, dom_bits, dom_count,
                                  spt, sln, take, 1, w.search)
    assert (e_pt[:32] == np.array([0, 1, 2])).all()
    # a round-1 contact without a link is not extended
    sln2 = sln.copy()
    sln2[:, 0, 1] = -1
    e_pt, _, _ = oracle.extend(w.hand, w.field, bits, w.obj.pts, w.obj.nrm, w.poses, dom_bits, dom_count,
                               spt, sln2, take, 1, w.search)
    assert (e_pt[:, 0] == -1).all() and (e_pt[:, 1:] >= 0).all()
    # k1 + k_add above the finger count is refused
    with pytest.raises(ValueError):
        oracle.extend(w.hand, w.field, bits, w.obj.pts, w.obj.nrm, w.poses, dom_bits, dom_count,
                      spt, sln, take, 4, w.search)


def test_extension_is_keyed_by_global_indices(c3k):
    w, ref, Q, spt, sln, V = c3k
    take = _take(spt, sln, V)
    full = oracle.extend(w.hand, w.field, ref["bits"], w.obj.pts, w.obj.nrm, w.poses, Q["dom_bits"],
                         Q["dom_count"], spt, sln, take, 2, w.search, request_id=4)
    # a subset of the sets
    sub = take.copy()
    sub[::2] = 0
    part = oracle.extend(w.hand, w.field, ref["bits"], w.obj.pts, w.obj.nrm, w.poses, Q["dom_bits"],
                         Q["dom_count"], spt, sln, sub, 2, w.search, request_id=4)
    on = sub.astype(bool)
    assert np.array_equal(part[0][on], full[0][on]) and np.array_equal(part[1][on], full[1][on])
    # one pose alone at its global offset
    g = 37
    sp_g = dataclasses.replace(w.search, pose_offset=g)
    one = oracle.extend(w.hand, w.field, ref["bits"], w.obj.pts, w.obj.nrm, w.poses[g:g + 1],
                        Q["dom_bits"][g:g + 1], Q["dom_count"][g:g + 1], spt[g:g + 1], sln[g:g + 1],
                        take[g:g + 1], 2, sp_g, request_id=4)
    assert np.array_equal(one[0][0], full[0][g]) and np.array_equal(one[1][0], full[1][g])
    # another request id gives other sets
    other = oracle.extend(w.hand, w.field, ref["bits"], w.obj.pts, w.obj.nrm, w.poses, Q["dom_bits"],
                          Q["dom_count"], spt, sln, take, 2, w.search, request_id=5)
    ext = full[0][..., 0] >= 0
    assert (other[0][ext] != full[0][ext]).any()
