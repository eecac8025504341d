"""Pins of the hand self-collision oracle (Sec. 5.6 postprocessing):

* the closed-form segment distance against brute force over a fine
  parameter grid, within the grid's error bound, and against exact special
  cases (crossing, parallel, collinear, point-like segments);
* the self-penetration of a hand against brute force over every pair of links
  of different fingers;
* realize with the filter on: depth = max(object, self) penetration, and
  validity never gained by turning the filter on.
"""
import dataclasses

import numpy as np
import pytest

import oracle
import synth


def _brute(p1, q1, p2, q2, n=401):
    s = np.linspace(0.0, 1.0, n)
    a = p1[None, :] + s[:, None] * (q1 - p1)[None, :]
    b = p2[None, :] + s[:, None] * (q2 - p2)[None, :]
    d = np.sqrt(((a[:, None, :] - b[None, :, :]) ** 2).sum(-1))
    # grid bound: each parameter is within 1/(2(n-1)) of the optimum
    bound = (np.linalg.norm(q1 - p1) + np.linalg.norm(q2 - p2)) / (2 * (n - 1))
    return d.min(), bound


def test_segment_distance_against_brute_force():
    rng = np.random.default_rng(0)
    for _ in range(150):
        p1, q1, p2, q2 = rng.uniform(-0.05, 0.05, size=(4, 3))
        d = oracle.segment_distance(p1, q1, p2, q2)
        b, bound = _brute(p1, q1, p2, q2)
        assert d <= b + 1e-12          # the closed form is a true minimum
        assert b - d <= bound + 1e-12


def test_segment_distance_special_cases():
    x, y, z = np.eye(3)
    o = np.zeros(3)
    # crossing segments at distance 0.3 along z
    assert oracle.segment_distance(-x, x, -y + 0.3 * z, y + 0.3 * z) == pytest.approx(0.3, abs=1e-15)
    # parallel, overlapping in extent: the separation
    assert oracle.segment_distance(o, x, 0.2 * y, x + 0.2 * y) == pytest.approx(0.2, abs=1e-15)
    # collinear, disjoint: the gap between the ends
    assert oracle.segment_distance(o, x, 1.5 * x, 3 * x) == pytest.approx(0.5, abs=1e-15)
    # a point against a segment, and two points
    assert oracle.segment_distance(0.5 * x + 0.25 * y, 0.5 * x + 0.25 * y, o, x) == pytest.approx(0.25, abs=1e-15)
    assert oracle.segment_distance(o, o, z, z) == pytest.approx(1.0, abs=1e-15)
    # endpoints beyond each other's extent
    assert oracle.segment_distance(o, x, 2 * x + y, 3 * x + y) == pytest.approx(np.sqrt(2.0), abs=1e-15)


@pytest.mark.parametrize("name", ["c1", "c3"])
def test_self_penetration_against_brute_force(name):
    w = synth.workload(name, n_poses=1, with_sdf=False)
    H = w.hand
    rng = np.random.default_rng(1)
    for _ in range(8):
        q = rng.uniform(H.limits[:, 0], H.limits[:, 1])
        T = oracle.fk(H, q)
        caps = []
        for l in range(H.n_joints):
            M = T[l].reshape(3, 4)
            c = H.capsule[l].astype(np.float64)
            caps.append((M[:, :3] @ c[:3] + M[:, 3], M[:, :3] @ c[3:6] + M[:, 3], c[6]))
        best, slack = -np.inf, 0.0
        for a in range(H.n_joints):
            for b in range(a + 1, H.n_joints):
                if H.joint_finger[a] == H.joint_finger[b]:
                    continue
                d, bound = _brute(caps[a][0], caps[a][1], caps[b][0], caps[b][1], n=201)
                pen = caps[a][2] + caps[b][2] - d
                if pen > best:
                    best, slack = pen, bound
        got = oracle.self_penetration(H, q)
        assert got >= best - 1e-12 and got - best <= slack + 1e-12


def test_realize_with_the_filter():
    w = synth.workload("c1", n_poses=128, with_sdf=True)
    fld = oracle.build_field(w.hand, w.field, witness=True, flags=False)
    Q = oracle.query(w.hand, w.field, fld["bits"], w.obj.pts, w.obj.nrm, w.poses, flags=False)
    spt, sln = oracle.draw(w.hand, w.field, fld["bits"], w.obj.pts, w.obj.nrm, w.poses, Q["dom_bits"],
                           Q["dom_count"], w.search)
    V = oracle.verdicts(w.obj.pts, w.obj.nrm, spt, w.search)
    acc = oracle.compact(V["verdict"])
    assert len(acc) > 0
    k = w.search.k
    args = (w.hand, w.field, fld["wit"], w.sdf, w.obj.pts, w.obj.nrm, w.poses, spt.reshape(-1, k),
            sln.reshape(-1, k), w.search, acc)
    R0 = oracle.realize(*args, w.ik)
    R1 = oracle.realize(*args, dataclasses.replace(w.ik, self_collision=1))
    np.testing.assert_array_equal(R0["q"], R1["q"])
    assert np.all(R1["depth"] >= R0["depth"])
    assert np.all(R1["valid"] <= R0["valid"])
    # depth = max(object, self) at the final configurations
    for a in range(len(acc)):
        sp = oracle.self_penetration(w.hand, R0["q"][a])
        assert R1["depth"][a] == pytest.approx(max(R0["depth"][a], sp), abs=1e-12)
