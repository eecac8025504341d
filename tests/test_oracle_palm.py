"""Pins of the static-link (palm) contact oracle (Sec. 5.1: the object placed
against the palm with some probability, placements that penetrate rejected,
the palm contact carried into the search):

* every palm placement puts its object point on its palm sample with opposed
  normals (the selection words recomputed from Philox, pinned by its
  known-answer vectors); the other poses are untouched; the selection rate is
  the probability (binomial bound);
* rejection agrees with the palm capsules' penetration recomputed with scipy's
  RegularGridInterpolator (an independent trilinear interpolation); a ball
  resting on the palm is never rejected; the tool sometimes is;
* a palm contact completes a grasp: one finger contact nearly antipodal to the
  palm contact on a sphere balances (t* = 0, the chord inside both friction
  cones), the finger contact alone never does; palm_pt = -1 everywhere gives
  the plain verdicts;
* draws skip rejected placements and are otherwise unchanged; Alg. 2 with the
  palm keeps every point at a vanishing step (t* = the palm verdicts'), and
  over a batch it raises acceptance and lowers the mean t*.
"""
import math

import numpy as np
import pytest
from scipy.interpolate import RegularGridInterpolator

import oracle
import synth


def _words(seed, g, rid=0):
    key = (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    return np.concatenate([oracle.philox((g, b, 17, rid), key) for b in range(2)]).astype(np.uint64)


def _interp(sdf):
    G, h = sdf.dims, float(np.float32(sdf.h))
    o = sdf.origin.astype(np.float64)
    ax = [o[a] + h * np.arange(G) for a in range(3)]
    return RegularGridInterpolator(ax, np.transpose(sdf.values.astype(np.float64), (2, 1, 0)),
                                   bounds_error=False, fill_value=np.inf)


@pytest.fixture(scope="module")
def c3():
    return synth.workload("c3", n_poses=400, with_sdf=True, samples=1024, n_points=8192)


def test_palm_placement_geometry_and_rate(c3):
    w = c3
    palm = synth.palm_for("c3")
    seed, prob = 21, 0.4
    r = oracle.place_palm(palm, w.sdf, w.obj.pts, w.obj.nrm, w.poses, prob, 0.002, seed)
    P = len(w.poses)
    sel = 0
    for g in range(P):
        wd = _words(seed, g)
        u0 = (int(wd[0]) >> 8) / 2 ** 24
        if not u0 < prob:
            assert r["palm_pt"][g] == -1
            np.testing.assert_array_equal(r["poses"][g], w.poses[g].astype(np.float64))
            continue
        sel += 1
        js = int((wd[1] * np.uint64(palm.surf.shape[0])) >> np.uint64(32))
        i = int((wd[2] * np.uint64(w.obj.n)) >> np.uint64(32))
        assert r["palm_pt"][g] in (i, -2)
        M = r["poses"][g].reshape(3, 4)
        R, t = M[:, :3], M[:, 3]
        np.testing.assert_allclose(R.T @ R, np.eye(3), atol=1e-12)
        np.testing.assert_allclose(R @ w.obj.pts[i].astype(np.float64) + t, palm.surf[js, :3], atol=1e-12)
        n = w.obj.nrm[i].astype(np.float64)
        np.testing.assert_allclose(R @ (n / np.linalg.norm(n)), -palm.surf[js, 3:].astype(np.float64),
                                   atol=1e-12)
    assert abs(sel - prob * P) <= 5 * math.sqrt(P * prob * (1 - prob))


def test_rejection_is_the_capsule_penetration(c3):
    w = c3
    palm = synth.palm_for("c3")
    margin = 0.002
    r = oracle.place_palm(palm, w.sdf, w.obj.pts, w.obj.nrm, w.poses, 1.0, margin, 5)
    f = _interp(w.sdf)
    rejected = 0
    for g in range(len(w.poses)):
        M = r["poses"][g].reshape(3, 4)
        R, t = M[:, :3], M[:, 3]
        depth = -np.inf
        for c in palm.caps.astype(np.float64):
            L = np.linalg.norm(c[3:6] - c[:3])
            m = max(2, int(math.ceil(L / 1e-3)) + 1)
            x = c[:3] + np.linspace(0, 1, m)[:, None] * (c[3:6] - c[:3])
            y = (x - t) @ R                                 # R^T (x - t), row-wise
            depth = max(depth, float(np.max(c[6] - f(y))))
        if r["pflag"][g]:
            continue
        assert (r["palm_pt"][g] == -2) == (depth > margin), (g, depth)
        rejected += depth > margin
    assert 0 < rejected < len(w.poses)        # the tool sometimes reaches into the palm


def test_a_ball_on_the_palm_is_never_rejected():
    w = synth.workload("c1", n_poses=200, with_sdf=True)
    r = oracle.place_palm(synth.palm_for("c1"), w.sdf, w.obj.pts, w.obj.nrm, w.poses, 1.0, 0.002, 3)
    assert (r["palm_pt"] >= 0).all()


def test_palm_contact_completes_an_antipodal_grasp():
    w = synth.workload("c1", n_poses=1, with_sdf=False)
    pts, nrm = w.obj.pts, w.obj.nrm
    sp = w.search
    a = 0
    b = int(np.argmin(nrm @ nrm[a]))                    # nearest to antipodal
    chord = (pts[b] - pts[a]).astype(np.float64)
    chord /= np.linalg.norm(chord)
    assert math.acos(-chord @ nrm[a]) < math.atan(sp.mu) and math.acos(chord @ nrm[b]) < math.atan(sp.mu)
    one = np.array([[[a]]], np.int32)
    V = oracle.verdicts_palm(pts, nrm, one, np.array([b], np.int32), sp)
    assert V["verdict"][0] == 1 and V["tstar"][0] == pytest.approx(0.0, abs=1e-12)
    import dataclasses
    alone = oracle.verdicts(pts, nrm, one, dataclasses.replace(sp, k=1))
    assert alone["verdict"][0] == 0 and alone["tstar"][0] > 0.1
    # without palm contacts the palm verdicts are the plain ones
    rng = np.random.default_rng(0)
    sets = rng.integers(0, w.obj.n, size=(6, 5, sp.k)).astype(np.int32)
    V0 = oracle.verdicts(pts, nrm, sets, sp)
    V1 = oracle.verdicts_palm(pts, nrm, sets, np.full(6, -1, np.int32), sp)
    np.testing.assert_array_equal(V0["verdict"], V1["verdict"])
    np.testing.assert_array_equal(V0["tstar"], V1["tstar"])


def test_draws_and_optimisation_with_the_palm(c3):
    import dataclasses
    w = synth.workload("c3", n_poses=48, with_sdf=True, samples=2048, n_points=4096)
    palm = synth.palm_for("c3")
    r = oracle.place_palm(palm, w.sdf, w.obj.pts, w.obj.nrm, w.poses, 0.5, 0.002, 9)
    poses = r["poses"].astype(np.float32)
    pp = r["palm_pt"]
    assert (pp == -2).any() and (pp >= 0).any()
    fld = oracle.build_field(w.hand, w.field, flags=False)
    Q = oracle.query(w.hand, w.field, fld["bits"], w.obj.pts, w.obj.nrm, poses, flags=False)
    sp = dataclasses.replace(w.search, draws=16)
    s0, l0 = oracle.draw(w.hand, w.field, fld["bits"], w.obj.pts, w.obj.nrm, poses, Q["dom_bits"],
                         Q["dom_count"], sp)
    s1, l1 = oracle.draw(w.hand, w.field, fld["bits"], w.obj.pts, w.obj.nrm, poses, Q["dom_bits"],
                         Q["dom_count"], sp, palm_pt=pp)
    assert (s1[pp == -2] == -1).all()
    np.testing.assert_array_equal(s1[pp != -2], s0[pp != -2])
    np.testing.assert_array_equal(l1[pp != -2], l0[pp != -2])
    V = oracle.verdicts_palm(w.obj.pts, w.obj.nrm, s1, pp, sp)
    tiny = dataclasses.replace(sp, opt_outer=1, opt_inner=4, opt_sigma=1e-9)
    O = oracle.optimize(w.obj.pts, w.obj.nrm, Q["dom_bits"], s1, tiny, w.hand.n_fingers,
                        dom_count=Q["dom_count"], palm_pt=pp)
    np.testing.assert_array_equal(O["set_pt"], s1)
    ok = ~np.isnan(V["tstar"])
    np.testing.assert_allclose(O["tstar"][ok], V["tstar"][ok], atol=1e-12)
    opt = dataclasses.replace(sp, opt_outer=1, opt_inner=4, opt_sigma=0.004)
    O2 = oracle.optimize(w.obj.pts, w.obj.nrm, Q["dom_bits"], s1, opt, w.hand.n_fingers,
                         dom_count=Q["dom_count"], palm_pt=pp)
    ok2 = ok & ~np.isnan(O2["tstar"])
    # the current point is not itself a candidate, so single sets may get worse;
    # over the batch the acceptance rises and the mean t* falls
    assert O2["verdict"][ok2].sum() >= V["verdict"][ok2].sum()
    assert O2["tstar"][ok2].mean() < V["tstar"][ok2].mean()



def test_placement_flags_and_the_other_branch():
    """Flag bits name their cause; the selected point is recorded for every
    selected pose; flipping the rotation branch changes only poses whose
    alignment cosine lies in the branch band.  A one-point object whose normal
    meets the (upward) palm normals at a cosine inside the band: both branches
    put the point onto the palm sample with the normals opposed, in two
    different rotations."""
    w = synth.workload("c3", n_poses=512, samples=4096, with_sdf=True)
    palm = synth.palm_for("c3")
    r = oracle.place_palm(palm, w.sdf, w.obj.pts, w.obj.nrm, w.poses, 0.5, 0.002, 5)
    f = oracle.place_palm(palm, w.sdf, w.obj.pts, w.obj.nrm, w.poses, 0.5, 0.002, 5, flip=True)
    assert set(np.unique(r["pflag"])) <= {0, 1, 2, 3}
    sel = r["sel_pt"] >= 0
    kept = r["palm_pt"] >= 0
    assert ((r["palm_pt"] != -1) == sel).all() and (r["palm_pt"][kept] == r["sel_pt"][kept]).all()
    same = (r["poses"] == f["poses"]).all(1)
    assert (same | ((r["pflag"] & 1) != 0)).all()
    # the crafted point: cosine of its normal with b = -(palm normal) = -z is -0.9999 + 3e-6
    c = -0.9999 + 3e-6
    a = np.array([[np.sqrt(1 - c * c), 0.0, -c]], np.float32)
    pt = np.array([[0.0, 0.0, 0.04]], np.float32)
    poses = np.tile(np.eye(3, 4, dtype=np.float32).reshape(1, 12), (64, 1))
    r = oracle.place_palm(palm, w.sdf, pt, a, poses, 1.0, 0.002, 5)
    f = oracle.place_palm(palm, w.sdf, pt, a, poses, 1.0, 0.002, 5, flip=True)
    assert ((r["pflag"] & 1) != 0).all()
    an = a[0].astype(np.float64) / np.linalg.norm(a[0])
    for B in (r, f):
        for g in range(len(poses)):
            M = B["poses"][g].reshape(3, 4)
            assert abs(np.linalg.det(M[:, :3]) - 1) < 1e-9   # 1 / (1 + c) amplifies the rounding
            assert np.allclose(M[:, :3] @ an, [0, 0, -1], atol=1e-9)
    assert not np.allclose(r["poses"], f["poses"], atol=1e-3)
