"""Pins of the cone-query oracle (the theta_hit test of Sec. 4.3 over the
field's bin centres):

* cos_hit above 1 hits nothing; cos_hit = -1 hits exactly where the finger's
  voxel holds any bit (brute-force occupancy in NumPy);
* once the cone exceeds the bins' covering radius it contains the
  nearest-bin domain (every direction is that close to its nearest centre);
* domains grow monotonically as the cone widens.
"""
import math

import numpy as np
import pytest

import oracle
import synth


@pytest.fixture(scope="module")
def c1():
    w = synth.workload("c1", n_poses=24)
    ref = oracle.build_field(w.hand, w.field, flags=False)
    return w, ref["bits"]


def _unpack(words, n):
    return np.unpackbits(np.ascontiguousarray(words).view(np.uint8), axis=-1, bitorder="little")[..., :n].astype(bool)


def test_empty_and_full_cones(c1):
    w, bits = c1
    N = w.obj.n
    none = oracle.query_cone(w.hand, w.field, bits, w.obj.pts, w.obj.nrm, w.poses, 1.5)
    assert none["dom_count"].sum() == 0
    full = oracle.query_cone(w.hand, w.field, bits, w.obj.pts, w.obj.nrm, w.poses, -1.0)
    # brute-force occupancy: voxel of x in finger f's window holds any bit of any of f's links
    G, h = w.field.grid, float(w.field.h)
    gf = np.asarray(w.field.grid_frame, np.float64).reshape(-1, 3, 4)
    J = w.hand.n_joints
    occ = bits.reshape(J, G, G, G, -1).any(axis=-1)
    got = _unpack(full["dom_bits"], N)
    for g in range(len(w.poses)):
        P = w.poses[g].astype(np.float64).reshape(3, 4)
        x = w.obj.pts.astype(np.float64) @ P[:, :3].T + P[:, 3]
        for f in range(w.hand.n_fingers):
            u = (x - gf[f, :, 3]) @ gf[f, :, :3] / h
            v = np.floor(u).astype(int)
            inside = ((v >= 0) & (v < G)).all(axis=1)
            want = np.zeros(N, bool)
            links = np.flatnonzero(w.hand.joint_finger == f)
            vi = v[inside]
            want[inside] = occ[links][:, vi[:, 2], vi[:, 1], vi[:, 0]].any(axis=0)
            flag = _unpack(full["dom_flag"][g, f], N)
            assert np.array_equal(got[g, f][~flag], want[~flag])


def test_wide_cone_contains_the_nearest_bin_domain(c1):
    w, bits = c1
    B = w.field.bins
    cb = oracle.bin_centers(B)
    rng = np.random.default_rng(0)
    d = rng.normal(size=(200000, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    cover = math.acos(np.clip((d @ cb.T).max(axis=1).min(), -1, 1))   # covering radius (sampled)
    cone = oracle.query_cone(w.hand, w.field, bits, w.obj.pts, w.obj.nrm, w.poses, math.cos(cover + 0.02))
    nb = oracle.query(w.hand, w.field, bits, w.obj.pts, w.obj.nrm, w.poses)
    fl = (cone["dom_flag"] | nb["dom_flag"])
    assert ((nb["dom_bits"] & ~cone["dom_bits"]) & ~fl).sum() == 0


def test_domains_grow_with_the_cone(c1):
    w, bits = c1
    prev = None
    for deg in (5, 15, 30, 60):
        r = oracle.query_cone(w.hand, w.field, bits, w.obj.pts, w.obj.nrm, w.poses, math.cos(math.radians(deg)))
        if prev is not None:
            assert ((prev["dom_bits"] & ~r["dom_bits"]) & ~(prev["dom_flag"] | r["dom_flag"])).sum() == 0
            assert r["dom_count"].sum() >= prev["dom_count"].sum()
        prev = r
