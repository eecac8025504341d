"""Pins of the oracle's field construction, contact query and draws:
brute-force enumeration on tiny inputs, the closed-form reach of a planar
2-link finger, exact 90-degree rotation and translation invariance, and an
independent NumPy select / chi-square test of the draws.  CPU only."""
import math

import numpy as np
import pytest
from scipy.spatial import cKDTree

import oracle
import synth
from tests.test_oracle_kinematics import closed_form_tip, planar_2r_hand


def _fp(G, h, B, S, origin, R=np.eye(3), seed=0):
    gf = np.zeros((1, 12), np.float32)
    gf[0] = synth._pack34(R, np.asarray(origin, np.float64))
    return synth.FieldParams(samples=S, seed=seed, grid=G, h=h, bins=B, grid_frame=gf)


def _unpack(words, n):
    """uint32 bit words [..., W] -> bool [..., n] (bit i%32 of word i/32)."""
    b = np.unpackbits(words.view(np.uint8), axis=-1, bitorder="little")
    return b[..., :n].astype(bool)


def test_field_and_query_match_brute_force_enumeration():
    """Every (pose, point) is hit iff some (joint sample, link, surface
    sample) contact vector lands in the same voxel and normal bin (no table)."""
    h = planar_2r_hand(tip_only=False)
    G, hv, B, S = 16, 0.008, 32, 64
    # a rotated window (catches a transposed grid rotation)
    cz, sz, cx, sx = math.cos(0.4), math.sin(0.4), math.cos(0.2), math.sin(0.2)
    Rw = np.array([[cz, -sz, 0], [sz, cz, 0], [0, 0, 1.0]]) @ np.array([[1.0, 0, 0], [0, cx, -sx], [0, sx, cx]])
    centre = np.array([0.0013, -0.045, 0.025])
    fp = _fp(G, hv, B, S, origin=centre - Rw @ np.full(3, 0.5 * G * hv), R=Rw)
    fld = oracle.build_field(h, fp)
    # object: small sphere inside the reach, a few poses around it
    obj = synth.sphere_object(0.02, 96)
    rng = np.random.default_rng(5)
    poses = np.zeros((6, 12), np.float32)
    for g in range(6):
        R = synth._quat_to_R(synth._shoemake(rng.uniform(size=3)))
        t = np.array([0.0, -0.05, 0.04]) + rng.uniform(-0.01, 0.01, size=3)
        poses[g] = synth._pack34(R, t)
    Q = oracle.query(h, fp, fld["bits"], obj.pts, obj.nrm, poses)

    c = oracle.bin_centers(B)
    tree = cKDTree(c)
    Rg = fp.grid_frame[0].reshape(3, 4)[:, :3].astype(np.float64)
    og = fp.grid_frame[0].reshape(3, 4)[:, 3].astype(np.float64)
    hh = float(np.float32(hv))

    def vox(x):
        u = (x - og) @ Rg / hh
        inside = np.all((u >= 0) & (u < G), axis=-1)
        return np.floor(u).astype(np.int64), inside

    # enumerate every contact vector of the finger
    keys = set()
    for s in range(S):
        q = np.zeros(h.n_joints)
        q[h.finger_joints(0)] = oracle.joint_sample(h, fp.seed, 0, s)
        T = oracle.fk(h, q)
        for l in range(h.n_joints):
            Tl = T[l].reshape(3, 4)
            sp = h.surf[l].astype(np.float64)
            x = sp[:, :3] @ Tl[:, :3].T + Tl[:, 3]
            nu = sp[:, 3:] @ Tl[:, :3].T
            v, ins = vox(x)
            _, b = tree.query(nu / np.linalg.norm(nu, axis=1, keepdims=True))
            for vv, bb, ok in zip(v, b, ins):
                if ok:
                    keys.add((tuple(vv), int(bb)))
    assert len(keys) > 50
    n = obj.n
    got = _unpack(Q["dom_bits"][:, 0, :], n)
    flag = _unpack(Q["dom_flag"][:, 0, :], n)
    p = obj.pts.astype(np.float64)
    nn = obj.nrm.astype(np.float64)
    n_hits = 0
    for g in range(poses.shape[0]):
        P = poses[g].reshape(3, 4).astype(np.float64)
        x = p @ P[:, :3].T + P[:, 3]
        qd = -(nn @ P[:, :3].T)  # contact surface representation: negated normal
        v, ins = vox(x)
        _, b = tree.query(qd / np.linalg.norm(qd, axis=1, keepdims=True))
        want = np.array([bool(ok) and ((tuple(vv), int(bb)) in keys) for vv, bb, ok in zip(v, b, ins)])
        n_hits += want.sum()
        mism = (want != got[g]) & ~flag[g]
        assert not mism.any(), (g, np.flatnonzero(mism))
        assert Q["dom_count"][g, 0] == got[g].sum()
    assert n_hits > 0


def test_field_closed_form_reach_of_planar_two_link_finger():
    """Marked voxels and bins of the fingertip table agree with the analytic
    reach of a planar 2R finger: tip = base + L1 e(q1) + L2 e(q1+q2), tip
    normal along the distal link, q in [0, 1.5]^2."""
    L1, L2, lo, hi = 0.05, 0.04, 0.0, 1.5
    h = planar_2r_hand(L1, L2, lo=lo, hi=hi)
    G, hv, B, S = 32, 0.004, 32, 65536
    origin = np.array([-0.0641, -0.095, -0.0375])
    fp = _fp(G, hv, B, S, origin)
    fld = oracle.build_field(h, fp, flags=True)
    hh = float(np.float32(hv))
    og = fp.grid_frame[0].reshape(3, 4)[:, 3].astype(np.float64)
    bits = _unpack(fld["bits"][1], B)   # distal link table [G^3, B]
    assert fld["stats"][2] == 0          # window covers the whole reach
    marked_vox = np.flatnonzero(bits.any(axis=1))
    # dense lattice of the closed form
    m = 1500
    q1, q2 = np.meshgrid(np.linspace(lo, hi, m), np.linspace(lo, hi, m), indexing="ij")
    y, z, phi = closed_form_tip(q1.ravel(), q2.ravel(), L1, L2)
    iy = np.floor((y - og[1]) / hh).astype(np.int64)
    iz = np.floor((z - og[2]) / hh).astype(np.int64)
    ix = int(np.floor((0.0 - og[0]) / hh))
    dense_vox = (iz * G + iy) * G + ix
    dense_set = set(np.unique(dense_vox).tolist())
    # (1) soundness: every marked voxel is reached by the closed form
    outside = [v for v in marked_vox.tolist() if v not in dense_set]
    assert len(outside) <= max(1, len(marked_vox) // 200), outside[:10]
    # (2) completeness: voxels whose whole square lies well inside the reach
    rho_lo = math.sqrt(L1 ** 2 + L2 ** 2 + 2 * L1 * L2 * math.cos(hi))
    rho_hi = L1 + L2

    def inside(yy, zz, margin):
        rho = np.hypot(yy, zz)
        ok = (rho >= rho_lo + margin) & (rho <= rho_hi - margin)
        c2 = np.clip((rho ** 2 - L1 ** 2 - L2 ** 2) / (2 * L1 * L2), -1, 1)
        qq2 = np.arccos(c2)
        alpha = np.arctan2(L2 * np.sin(qq2), L1 + L2 * np.cos(qq2))
        theta = np.arctan2(-yy, zz)
        ang_margin = margin / np.maximum(rho, 1e-9)
        ok &= (theta - alpha >= lo + ang_margin) & (theta - alpha <= hi - ang_margin)
        return ok & (qq2 >= lo) & (qq2 <= hi)
    deep = []
    for vy in range(G):
        for vz in range(G):
            cy, cz = og[1] + (vy + 0.5) * hh, og[2] + (vz + 0.5) * hh
            if inside(np.array([cy]), np.array([cz]), hh * math.sqrt(2) / 2 + 0.001)[0]:
                deep.append((vz * G + vy) * G + ix)
    assert len(deep) > 20
    missing = [v for v in deep if not bits[v].any()]
    assert not missing, missing[:10]
    # (3) bins: marked bins of a voxel are bins of tip directions reaching it
    c = oracle.bin_centers(B)
    tree = cKDTree(c)
    allowed = {}
    for dphi in (-0.004, 0.0, 0.004):
        d = np.stack([np.zeros_like(phi), -np.sin(phi + dphi), np.cos(phi + dphi)], axis=1)
        _, bb = tree.query(d)
        for v, b in zip(dense_vox.tolist(), bb.tolist()):
            allowed.setdefault(v, set()).add(b)
    bad = 0
    for v in marked_vox.tolist():
        for b in np.flatnonzero(bits[v]).tolist():
            if b not in allowed.get(v, ()):
                bad += 1
    assert bad <= max(1, int(0.005 * bits.sum())), bad


@pytest.fixture(scope="module")
def c1_small():
    w = synth.workload("c1", n_poses=48)
    fld = oracle.build_field(w.hand, w.field, witness=False)
    Q = oracle.query(w.hand, w.field, fld["bits"], w.obj.pts, w.obj.nrm, w.poses)
    return w, fld, Q


def test_query_exact_90_degree_rotation_invariance(c1_small):
    """(R0 p, R0 n) with pose R R0^T gives the same domains (R0 = 90 deg about z)."""
    w, fld, Q = c1_small
    R0 = np.array([[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
    p2 = (w.obj.pts.astype(np.float64) @ R0.T).astype(np.float32)
    n2 = (w.obj.nrm.astype(np.float64) @ R0.T).astype(np.float32)
    P = w.poses.reshape(-1, 3, 4).astype(np.float64).copy()
    P[:, :, :3] = P[:, :, :3] @ R0.T
    Q2 = oracle.query(w.hand, w.field, fld["bits"], p2, n2, P.reshape(-1, 12).astype(np.float32))
    fl = Q["dom_flag"] | Q2["dom_flag"]
    assert ((Q["dom_bits"] ^ Q2["dom_bits"]) & ~fl).sum() == 0
    assert Q["dom_count"].sum() > 0


def test_query_translation_invariance(c1_small):
    """Moving the object frame by d and the pose by -R d leaves domains unchanged."""
    w, fld, Q = c1_small
    d = np.array([0.01, -0.02, 0.005])
    p2 = (w.obj.pts.astype(np.float64) + d).astype(np.float32)
    P = w.poses.reshape(-1, 3, 4).astype(np.float64).copy()
    P[:, :, 3] -= P[:, :, :3] @ d
    Q2 = oracle.query(w.hand, w.field, fld["bits"], p2, w.obj.nrm, P.reshape(-1, 12).astype(np.float32))
    fl = Q["dom_flag"] | Q2["dom_flag"]
    assert ((Q["dom_bits"] ^ Q2["dom_bits"]) & ~fl).sum() == 0


def _draw_words(seed, rid, g, d, n):
    out = []
    for blk in range((n + 3) // 4):
        out += list(oracle.philox([g, 4 * d + blk, 3, rid], [seed & 0xFFFFFFFF, seed >> 32]))
    return [int(x) for x in out[:n]]


def test_draws_match_independent_select(c1_small):
    """Drawn point j = floor(r * count / 2^32)-th set bit (NumPy select);
    empty domains give -1; the drawn link's table bit is set."""
    w, fld, Q = c1_small
    sp = w.search
    spt, sln = oracle.draw(w.hand, w.field, fld["bits"], w.obj.pts, w.obj.nrm, w.poses,
                           Q["dom_bits"], Q["dom_count"], sp)
    n, k = w.obj.n, sp.k
    dom = _unpack(Q["dom_bits"], n)
    n_valid = 0
    for g in range(w.poses.shape[0]):
        empty = (Q["dom_count"][g] == 0).any()
        for d in range(sp.draws):
            if empty:
                assert (spt[g, d] == -1).all() and (sln[g, d] == -1).all()
                continue
            n_valid += 1
            r = _draw_words(sp.seed, sp.request_id, g, d, 2 * k)
            for i in range(k):
                idx = np.flatnonzero(dom[g, i])
                j = (r[i] * len(idx)) >> 32
                assert spt[g, d, i] == idx[j]
                assert sln[g, d, i] in w.hand.finger_joints(i)
    assert n_valid > 0
    # drawn link's own table bit is set at the point's voxel and bin
    B, G = w.field.bins, w.field.grid
    tree = cKDTree(oracle.bin_centers(B))
    bits = _unpack(fld["bits"], B)
    hh = float(np.float32(w.field.h))
    for g, d in zip(*np.nonzero(spt[:, :, 0] >= 0)):
        P = w.poses[g].reshape(3, 4).astype(np.float64)
        for i in range(k):
            idx, l = spt[g, d, i], sln[g, d, i]
            x = P[:, :3] @ w.obj.pts[idx].astype(np.float64) + P[:, 3]
            qd = -(P[:, :3] @ w.obj.nrm[idx].astype(np.float64))
            F = w.field.grid_frame[i].reshape(3, 4).astype(np.float64)
            u = np.floor((x - F[:, 3]) @ F[:, :3] / hh).astype(int)
            _, b = tree.query(qd / np.linalg.norm(qd))
            assert bits[l, (u[2] * G + u[1]) * G + u[0], b]


def test_draw_uniformity_chi_square(c1_small):
    """The point draws are uniform over a domain (chi-square)."""
    w, fld, Q = c1_small
    g = int(np.flatnonzero((Q["dom_count"] > 0).all(axis=1))[0])
    sp = synth.SearchParams(draws=60000, k=w.search.k, mu=0.5, m_edges=8, eps=1e-3, seed=11)
    spt, _ = oracle.draw(w.hand, w.field, fld["bits"], w.obj.pts, w.obj.nrm, w.poses[g:g + 1],
                         Q["dom_bits"][g:g + 1], Q["dom_count"][g:g + 1], sp)
    cnt = int(Q["dom_count"][g, 0])
    vals, counts = np.unique(spt[0, :, 0], return_counts=True)
    assert len(vals) == cnt
    e = sp.draws / cnt
    chi2 = ((counts - e) ** 2 / e).sum()
    dof = cnt - 1
    assert chi2 < dof + 5 * math.sqrt(2 * dof)


def test_field_over_a_subset_of_joint_samples():
    """The cover restricted to a subset of joint samples is contained in the
    full cover (bits and sure bits), its smallest reaching sample is never
    below the full cover's, and the subset of every sample is the full cover."""
    w = synth.workload("c1", n_poses=8)
    full = oracle.build_field(w.hand, w.field, witness=True)
    ids = np.sort(np.random.default_rng(1).choice(w.field.samples, 500, replace=False))
    sub = oracle.build_field(w.hand, w.field, witness=True, sample_ids=ids)
    assert ((sub["bits"] & ~full["bits"]) == 0).all() and ((sub["sure"] & ~full["sure"]) == 0).all()
    assert (sub["bits"] != full["bits"]).any()
    h = sub["wit"] >= 0
    assert (full["wit"][h] <= sub["wit"][h]).all()
    assert np.isin(sub["wit"][h], ids).all()
    every = oracle.build_field(w.hand, w.field, witness=True, sample_ids=np.arange(w.field.samples))
    assert (every["bits"] == full["bits"]).all() and (every["wit"] == full["wit"]).all()
    with pytest.raises(ValueError):
        oracle.build_field(w.hand, w.field, sample_ids=[w.field.samples])
