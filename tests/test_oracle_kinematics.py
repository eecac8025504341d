"""Pins of the oracle's RNG, kinematics and normal bins against things other
than the oracle itself: published known-answer vectors, closed forms, finite
differences, a library nearest-neighbour search and the paper's worked
example.  CPU only."""
import math
import os

import numpy as np
import pytest
from scipy.spatial import cKDTree

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


def test_philox_known_answers():
    """Philox4x32-10 reproduces the known-answer vectors published with it."""
    for row in _read_golden("philox4x32_10_kat.txt"):
        v = [int(x, 16) for x in row]
        out = oracle.philox(v[0:4], v[4:6])
        assert [int(x) for x in out] == v[6:10]


def test_joint_samples_uniform_in_limits():
    """Joint samples lie in [lo, hi) and are uniform (chi-square, 16 cells)."""
    h = synth.hand_c2()
    lo, hi = h.limits[0].astype(np.float64)
    q = np.array([oracle.joint_sample(h, 7, 1, s)[2] for s in range(4000)])
    js = h.finger_joints(1)
    lo, hi = h.limits[js[2]].astype(np.float64)
    assert q.min() >= lo and q.max() < hi
    cnt, _ = np.histogram(q, bins=16, range=(lo, hi))
    chi2 = ((cnt - 250.0) ** 2 / 250.0).sum()
    assert chi2 < 40.0  # 15 dof: p ~ 5e-4
    # different fingers / seeds give different streams
    assert not np.allclose(oracle.joint_sample(h, 7, 0, 5), oracle.joint_sample(h, 7, 1, 5))
    assert not np.allclose(oracle.joint_sample(h, 7, 0, 5), oracle.joint_sample(h, 8, 0, 5))


def planar_2r_hand(L1=0.05, L2=0.04, r=0.006, lo=0.0, hi=1.5, tip_only=True):
    """One planar finger with two flexion joints about x, base at the origin,
    links along +z at q = 0; one surface sample per link at its tip, normal
    along the link."""
    h = synth._build_hand([{"base": (np.eye(3), np.zeros(3)),
                            "joints": [(synth.X_AX, L1, r, lo, hi), (synth.X_AX, L2, r, lo, hi)]}],
                          n_surf=4)
    if tip_only:
        surf = np.zeros((2, 1, 6), np.float32)
        for j, L in enumerate((L1, L2)):
            surf[j, 0] = (0.0, 0.0, L, 0.0, 0.0, 1.0)
        h.surf = surf
    return h


def closed_form_tip(q1, q2, L1=0.05, L2=0.04):
    """Planar 2R tip (y, z) and link-2 direction angle (rotation about +x)."""
    y = -L1 * np.sin(q1) - L2 * np.sin(q1 + q2)
    z = L1 * np.cos(q1) + L2 * np.cos(q1 + q2)
    return y, z, q1 + q2


def test_fk_planar_2r_closed_form():
    h = planar_2r_hand()
    rng = np.random.default_rng(1)
    for _ in range(20):
        q = rng.uniform(-2, 2, size=2)
        T = oracle.fk(h, q)
        tip = T[1].reshape(3, 4) @ np.array([0, 0, 0.04, 1.0])
        y, z, phi = closed_form_tip(q[0], q[1])
        assert np.allclose(tip, [0.0, y, z], atol=1e-12)
        d = T[1].reshape(3, 4)[:, 2]
        assert np.allclose(d, [0.0, -math.sin(phi), math.cos(phi)], atol=1e-12)


@pytest.mark.parametrize("hand_name", ["c1", "c2", "c3"])
def test_point_jacobian_matches_finite_differences(hand_name):
    """Eq. 8 (base-frame form) against central differences of FK."""
    h = {"c1": synth.hand_c1, "c2": synth.hand_c2, "c3": synth.hand_c3}[hand_name]()
    rng = np.random.default_rng(2)
    q = rng.uniform(h.limits[:, 0], h.limits[:, 1]).astype(np.float64)
    for f in range(h.n_fingers):
        js = h.finger_joints(f)
        for link in js:
            loc = np.array([0.003, -0.004, 0.01, 1.0])  # point fixed to the link
            x = oracle.fk(h, q)[link].reshape(3, 4) @ loc
            Jm = oracle.point_jacobian(h, f, int(link), q, x)
            eps = 1e-6
            for t, j in enumerate(js):
                qp, qm = q.copy(), q.copy()
                qp[j] += eps
                qm[j] -= eps
                xp = oracle.fk(h, qp)[link].reshape(3, 4) @ loc
                xm = oracle.fk(h, qm)[link].reshape(3, 4) @ loc
                assert np.allclose(Jm[:, t], (xp - xm) / (2 * eps), atol=1e-8)


@pytest.mark.parametrize("B", [32, 64, 256])
def test_bins_are_nearest_fibonacci_centres(B):
    """argmax <d, c_b> equals a KD-tree nearest-centre search (scipy)."""
    c = oracle.bin_centers(B)
    assert np.allclose(np.linalg.norm(c, axis=1), 1.0, atol=1e-14)
    assert np.allclose(c[:, 2], 1.0 - (2 * np.arange(B) + 1) / B)  # evenly spaced z
    rng = np.random.default_rng(3)
    d = rng.normal(size=(4000, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    _, nn = cKDTree(c).query(d)
    got = np.array([oracle.bin_of(B, v)[0] for v in d])
    gaps = np.array([oracle.bin_of(B, v)[2] for v in d])
    ok = gaps > 1e-9
    assert (got[ok] == nn[ok]).all()


def test_bin_cap_worked_example():
    """Sec. 4.3: 256 normal vectors give a cone half-angle of about 7 deg;
    the Fibonacci cells are near equal-area caps of that size."""
    for B, printed, tol in ([float(x) for x in r] for r in _read_golden("normal_bin_cap.txt")):
        B = int(B)
        theta = math.degrees(math.acos(1.0 - 2.0 / B))
        assert abs(theta - printed) < tol
        c = oracle.bin_centers(B)
        rng = np.random.default_rng(4)
        d = rng.normal(size=(200000, 3))
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        dist, nn = cKDTree(c).query(d)
        ang = 2.0 * np.degrees(np.arcsin(np.minimum(dist / 2.0, 1.0)))
        # equal areas: every cell holds ~1/B of uniform directions
        frac = np.bincount(nn, minlength=B) / d.shape[0]
        assert abs(frac.mean() - 1.0 / B) < 1e-12 and frac.std() * B < 0.15
        # a cap of half-angle theta has mean angular radius ~ 2/3 theta; a
        # non-circular cell of the same area has a slightly larger one
        assert 0.64 * theta < ang.mean() < 0.75 * theta
