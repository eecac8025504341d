"""Pins of the exhaustive-placement oracle (Sec. 5.1):

* the minimal rotation against scipy's rotation-vector construction (axis
  a x b, angle acos(a.b)) and, for (anti)parallel inputs, against its defining
  properties;
* each placed pose puts its object point on the chosen contact vector of the
  field with opposite normals, the contact vector recomputed independently
  with the joint sample and FK (each pinned elsewhere);
* the draws are uniform: fingers and object points by chi-square, roll angles
  by their first moments.
"""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation
from scipy.stats import chi2

import oracle
import synth


def test_rot_align_minimal_rotation():
    rng = np.random.default_rng(0)
    for _ in range(300):
        a, b = rng.normal(size=(2, 3))
        a /= np.linalg.norm(a)
        b /= np.linalg.norm(b)
        if a @ b <= -0.9999:
            continue
        R = oracle.rot_align(a, b)
        ax = np.cross(a, b)
        ang = math.atan2(np.linalg.norm(ax), a @ b)
        ref = Rotation.from_rotvec(ax / max(np.linalg.norm(ax), 1e-300) * ang).as_matrix()
        np.testing.assert_allclose(R, ref, atol=1e-12)


@pytest.mark.parametrize("c", [1.0, -1.0, -0.99999, -0.9999001, 0.0])
def test_rot_align_special_cases(c):
    rng = np.random.default_rng(1)
    a = rng.normal(size=3)
    a /= np.linalg.norm(a)
    u = np.cross(a, rng.normal(size=3))
    u /= np.linalg.norm(u)
    b = c * a + math.sqrt(max(0.0, 1 - c * c)) * u
    R = oracle.rot_align(a, b)
    np.testing.assert_allclose(R.T @ R, np.eye(3), atol=1e-12)
    assert np.linalg.det(R) == pytest.approx(1.0, abs=1e-12)
    np.testing.assert_allclose(R @ a, b, atol=1e-12)


def _draws(seed, g, n_fingers, samples, dof, n_surf, n_points):
    key = (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    w = np.concatenate([oracle.philox((g, b, 11, 0), key) for b in range(2)]).astype(np.uint64)
    f = int((w[0] * np.uint64(n_fingers)) >> np.uint64(32))
    s = int((w[1] * np.uint64(samples)) >> np.uint64(32))
    t = int((w[2] * np.uint64(dof[f])) >> np.uint64(32))
    j = int((w[3] * np.uint64(n_surf)) >> np.uint64(32))
    i = int((w[4] * np.uint64(n_points)) >> np.uint64(32))
    psi = 2 * math.pi * (int(w[5]) >> 8) / 2 ** 24
    return f, s, t, j, i, psi


@pytest.mark.parametrize("name", ["c1", "c3"])
def test_placement_puts_the_point_on_the_contact_vector(name):
    w = synth.workload(name, n_poses=1, with_sdf=False)
    H = w.hand
    seed = 77
    P = oracle.place_exhaustive(H, w.field, w.obj.pts, w.obj.nrm, 64, seed)["poses"]
    dof = H.dof
    firsts = [int(np.flatnonzero(H.joint_finger == f)[0]) for f in range(H.n_fingers)]
    for g in range(64):
        f, s, t, j, i, psi = _draws(seed, g, H.n_fingers, w.field.samples, dof, H.surf.shape[1], w.obj.n)
        q = np.zeros(H.n_joints)
        q[firsts[f]:firsts[f] + dof[f]] = oracle.joint_sample(H, w.field.seed, f, s)
        T = oracle.fk(H, q)[firsts[f] + t].reshape(3, 4)
        sf = H.surf[firsts[f] + t, j].astype(np.float64)
        x = T[:, :3] @ sf[:3] + T[:, 3]
        nu = T[:, :3] @ sf[3:]
        M = P[g].reshape(3, 4)
        R, tt = M[:, :3], M[:, 3]
        np.testing.assert_allclose(R.T @ R, np.eye(3), atol=1e-12)
        p, n = w.obj.pts[i].astype(np.float64), w.obj.nrm[i].astype(np.float64)
        np.testing.assert_allclose(R @ p + tt, x, atol=1e-12)
        np.testing.assert_allclose(R @ n / np.linalg.norm(n), -nu / np.linalg.norm(nu), atol=1e-12)


def test_placement_draws_are_uniform():
    w = synth.workload("c3", n_poses=1, with_sdf=False, n_points=512)
    H = w.hand
    n = 6000
    fs, idx, psis = [], [], []
    for g in range(n):
        f, s, t, j, i, psi = _draws(5, g, H.n_fingers, w.field.samples, H.dof, H.surf.shape[1], w.obj.n)
        fs.append(f)
        idx.append(i)
        psis.append(psi)
    cf = np.bincount(fs, minlength=H.n_fingers)
    e = n / H.n_fingers
    assert ((cf - e) ** 2 / e).sum() < chi2.ppf(0.999, H.n_fingers - 1)
    ci = np.bincount(np.array(idx) // 64, minlength=8)
    e = n / 8
    assert ((ci - e) ** 2 / e).sum() < chi2.ppf(0.999, 7)
    assert abs(np.mean(np.cos(psis))) < 5 / math.sqrt(2 * n) and abs(np.mean(np.sin(psis))) < 5 / math.sqrt(2 * n)
