"""Pins of the oracle's contact-set criterion (linearised-cone LP), IK and
penetration test: closed forms (antipodal pairs, the two-finger chord
condition with the m-gon cone, frictionless balance on a sphere), an
independent LP solver (scipy HiGHS), invariances and monotonicity, the
closed-form IK of a planar 2R finger, and the signed distance of a sphere.
CPU only."""
import math

import numpy as np
import pytest
from scipy.optimize import linprog
from scipy.spatial import ConvexHull

import oracle
import synth
from tests.test_oracle_kinematics import closed_form_tip, planar_2r_hand


def _highs_tstar(W):
    """min ||W^T g||_1, g >= 0, sum g = 1 with scipy's HiGHS (independent)."""
    n = W.shape[0]
    # variables g (n), s+ (6), s- (6)
    c = np.concatenate([np.zeros(n), np.ones(12)])
    A = np.zeros((7, n + 12))
    A[:6, :n] = W.T
    A[:6, n:n + 6] = -np.eye(6)
    A[:6, n + 6:] = np.eye(6)
    A[6, :n] = 1.0
    b = np.zeros(7)
    b[6] = 1.0
    res = linprog(c, A_eq=A, b_eq=b, bounds=[(0, None)] * (n + 12), method="highs")
    assert res.status == 0
    return res.fun


def _sphere_pts(dirs, R=0.04, c=(0.0, 0.0, 0.0)):
    d = np.asarray(dirs, np.float64)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return np.asarray(c) + R * d, d


def test_lp_matches_highs_on_random_sets():
    rng = np.random.default_rng(6)
    for trial in range(150):
        k = int(rng.integers(2, 6))
        p = rng.uniform(-0.05, 0.05, size=(k, 3))
        n = rng.normal(size=(k, 3))
        n /= np.linalg.norm(n, axis=1, keepdims=True)
        mu = float(rng.choice([0.0, 0.3, 0.5, 1.0]))
        W = oracle.wrench_matrix(p, n, mu, 8, 0.07)
        t, st, _ = oracle.lp_solve(W)
        assert st == 0
        assert abs(t - _highs_tstar(W)) < 1e-9


def test_antipodal_pair_balances_at_any_friction():
    for mu in (0.0, 0.1, 0.5):
        p, n = _sphere_pts([[1, 0.2, 0.3], [-1, -0.2, -0.3]])
        t, st = oracle.set_tstar(p, n, mu, 8, 0.04)
        assert st == 0 and t < 1e-12


def _mgon_radius(phi, mu, m):
    """Radius of the linearised cone's m-gon section at unit depth, in
    tangent direction phi (vertices at 2 pi e / m)."""
    w = 2 * math.pi / m
    phi_c = (math.floor(phi / w) + 0.5) * w
    return mu * math.cos(math.pi / m) / math.cos(phi - phi_c)


def test_two_finger_chord_condition():
    """Two contacts balance iff the chord lies in both (linearised) cones
    (Nguyen's two-finger condition) -- checked away from the boundary."""
    rng = np.random.default_rng(7)
    m, mu = 8, 0.5
    seen = [0, 0]
    for trial in range(800):
        p = rng.uniform(-0.05, 0.05, size=(2, 3))
        c = p[1] - p[0]
        c /= np.linalg.norm(c)
        if trial % 2:   # pinch-like: outward normals roughly along -c and +c
            n = np.stack([-c, c]) + 0.35 * rng.normal(size=(2, 3))
        else:
            n = rng.normal(size=(2, 3))
        n /= np.linalg.norm(n, axis=1, keepdims=True)
        margin = np.inf
        inside = False
        # force on contact 0 along +c (towards contact 1) or along -c
        for sgn in (1.0, -1.0):
            ok = True
            for i, dirn in ((0, sgn * c), (1, -sgn * c)):
                x, y = oracle.tangent_basis(n[i])
                depth = -(dirn @ n[i])       # component along -n_i (into the object)
                if depth <= 0:
                    ok = False
                    margin = min(margin, abs(depth))
                    continue
                tx, ty = dirn @ x / depth, dirn @ y / depth
                rho = math.hypot(tx, ty)
                phi = math.atan2(ty, tx) % (2 * math.pi)
                lim = _mgon_radius(phi, mu, m)
                ok &= rho <= lim
                margin = min(margin, abs(rho - lim))
            inside |= ok
        if margin < 0.02:
            continue
        t, st = oracle.set_tstar(p, n, mu, m, 0.07)
        assert st == 0
        assert (t < 1e-10) == inside, (trial, t, inside)
        seen[int(inside)] += 1
    assert seen[0] > 20 and seen[1] > 20


def test_frictionless_sphere_balance_is_zero_in_hull():
    """mu = 0 on a sphere: moments vanish and t* = 0 iff 0 in conv{n_i}."""
    rng = np.random.default_rng(8)
    seen = [0, 0]
    for trial in range(200):
        k = int(rng.integers(4, 7))
        p, n = _sphere_pts(rng.normal(size=(k, 3)))
        t, st = oracle.set_tstar(p, n, 0.0, 8, 0.04)
        hull = ConvexHull(n)
        # 0 inside iff all facet offsets are negative (strictly inside)
        off = hull.equations[:, 3]
        if np.min(np.abs(off)) < 1e-3:
            continue
        inside = bool((off < 0).all())
        assert (t < 1e-10) == inside
        seen[int(inside)] += 1
    assert seen[0] > 10 and seen[1] > 10


def test_lp_invariances_and_monotonicity():
    rng = np.random.default_rng(9)
    for trial in range(60):
        k = 4
        p = rng.uniform(-0.05, 0.05, size=(k, 3))
        n = rng.normal(size=(k, 3))
        n /= np.linalg.norm(n, axis=1, keepdims=True)
        t, _ = oracle.set_tstar(p, n, 0.5, 8, 0.07)
        # permutation of contacts
        perm = rng.permutation(k)
        t2, _ = oracle.set_tstar(p[perm], n[perm], 0.5, 8, 0.07)
        assert abs(t - t2) < 1e-10
        # balance (t* = 0) does not depend on the moment reference point
        t3, _ = oracle.set_tstar(p + rng.uniform(-0.1, 0.1, size=3), n, 0.5, 8, 0.07)
        assert (t < 1e-10) == (t3 < 1e-10)
        # more friction never breaks balance; more contacts never raise t*
        t4, _ = oracle.set_tstar(p, n, 0.8, 8, 0.07)
        if t < 1e-10:
            assert t4 < 1e-10
        t5, _ = oracle.set_tstar(p[:3], n[:3], 0.5, 8, 0.07)
        assert t <= t5 + 1e-12


def test_lp_pivot_cap_reports_undecided():
    p, n = _sphere_pts([[1, 0, 0], [-1, 0.1, 0], [0, 1, 0.2]])
    t, st = oracle.set_tstar(p, n, 0.5, 8, 0.04, max_pivots=0)
    assert st == 1


def test_ik_converges_to_closed_form_planar_2r():
    """DLS with tiny damping reaches the closed-form 2R solution (the
    fingertip cap point with the distal link direction as normal)."""
    L1, L2 = 0.05, 0.04
    h = planar_2r_hand(L1, L2, r=0.006, lo=-0.2, hi=1.7, tip_only=False)
    rng = np.random.default_rng(10)
    ik = synth.IKParams(iters=100, phase1=5, lam=1e-9, beta=0.01)
    for trial in range(10):
        qs = rng.uniform(0.2, 1.3, size=2)
        y, z, phi = closed_form_tip(qs[0], qs[1], L1, L2)
        d = np.array([0.0, -math.sin(phi), math.cos(phi)])
        p = np.array([0.0, y, z]) + 0.006 * d     # cap point along the link axis
        q0 = qs + rng.normal(0, 0.08, size=2)
        out = oracle.ik_finger(h, 0, 1, p, d, q0, ik)
        assert out["err"] < 1e-9 and out["ang"] < 1e-6
        # closed-form inverse kinematics of the tip (elbow branch of q0)
        rr = math.hypot(y, z)
        c2 = (rr ** 2 - L1 ** 2 - L2 ** 2) / (2 * L1 * L2)
        q2 = math.acos(max(-1.0, min(1.0, c2)))
        q1 = math.atan2(-y, z) - math.atan2(L2 * math.sin(q2), L1 + L2 * math.cos(q2))
        assert np.allclose(out["q"], [q1, q2], atol=1e-7)


def test_ik_standard_damping_reduces_error():
    """With the configured damping (lambda = 1e-2, 10 iterations) IK pulls a
    perturbed start onto a reachable contact."""
    h = synth.hand_c3()
    rng = np.random.default_rng(11)
    ik = synth.IKParams()
    errs0, errs = [], []
    for trial in range(20):
        f = int(rng.integers(0, h.n_fingers))
        js = h.finger_joints(f)
        l = int(js[-1])
        lo, hi = h.limits[js, 0].astype(float), h.limits[js, 1].astype(float)
        qs = rng.uniform(lo + 0.2, hi - 0.2)
        q = np.zeros(h.n_joints)
        q[js] = qs
        T = oracle.fk(h, q)[l].reshape(3, 4)
        cap = h.capsule[l].astype(np.float64)
        nl = np.array([0.0, 1.0, 0.0])
        p = T[:, :3] @ (cap[3:6] * 0.6 + cap[6] * nl) + T[:, 3]
        n = T[:, :3] @ nl
        q0 = np.clip(qs + rng.normal(0, 0.05, size=len(js)), lo, hi)
        e0 = oracle.ik_finger(h, f, l, p, n, q0, synth.IKParams(iters=0))["err"]
        out = oracle.ik_finger(h, f, l, p, n, q0, ik)
        errs0.append(e0)
        errs.append(out["err"])
    assert np.median(errs) < 0.3 * np.median(errs0)


def test_sdf_trilinear_on_sphere_closed_form():
    """Trilinear SDF of a sphere: error within h^2 kappa / 8 (+ rounding),
    +inf outside the grid."""
    R = 0.04
    sdf = synth.sdf_sphere(R)
    h = sdf.h
    rng = np.random.default_rng(12)
    y = rng.uniform(-0.05, 0.05, size=(2000, 3))
    got = np.array([oracle.sdf_eval(sdf, v) for v in y])
    want = np.linalg.norm(y, axis=1) - R
    rr = np.linalg.norm(y, axis=1)
    bound = 3 * h * h / (8 * np.maximum(rr, 1e-3)) + 1e-6
    assert (np.abs(got - want) <= bound).all()
    assert oracle.sdf_eval(sdf, np.array([1.0, 0, 0])) == math.inf


def test_penetration_depth_closed_form():
    """A single capsule at a known distance from a sphere: depth = r - (d - R)."""
    L, r = 0.03, 0.008
    h = synth._build_hand([{"base": (np.eye(3), np.zeros(3)),
                            "joints": [(synth.X_AX, L, r, -1.0, 1.0)]}], n_surf=4)
    R = 0.04
    sdf = synth.sdf_sphere(R)
    for dist in (0.045, 0.05, 0.06):
        # object centre on the -y side so the capsule axis (x=0..0, z in [0, L])
        # is closest at its ends
        pose = synth._pack34(np.eye(3), np.array([0.0, -dist, 0.5 * L])).astype(np.float32)
        depth = oracle.penetration(h, np.zeros(1), sdf, pose)
        want = r - (dist - R)
        assert abs(depth - want) < 3 * sdf.h ** 2 / (8 * R) + 1e-6
    assert oracle.axis_samples(h, 0) == math.ceil(round(L, 6) / 1e-3 - 1e-9) + 1 or oracle.axis_samples(h, 0) > 0


def _exact_tstar(W):
    """Exact optimum of the same LP in rational arithmetic (Bland's rule,
    no rounding): float inputs are converted exactly to fractions."""
    from fractions import Fraction as Fr
    n = W.shape[0]
    nv = n + 12
    A = [[Fr(0)] * (nv + 1) for _ in range(7)]
    for r in range(6):
        for c in range(n):
            A[r][c] = Fr(float(W[c, r]))
        A[r][n + r] = Fr(-1)
        A[r][n + 6 + r] = Fr(1)
    for c in range(n):
        A[6][c] = Fr(1)
    A[6][nv] = Fr(1)
    basis = [0] * 7
    for r in range(6):
        f = A[r][0]
        A[r] = [a - f * b for a, b in zip(A[r], A[6])]
        if A[r][nv] >= 0:
            basis[r] = n + 6 + r
        else:
            A[r] = [-a for a in A[r]]
            basis[r] = n + r
    cost = [Fr(0)] * n + [Fr(1)] * 12
    while True:
        red = [cost[j] - sum(cost[basis[r]] * A[r][j] for r in range(7)) for j in range(nv)]
        e = next((j for j in range(nv) if red[j] < 0), None)
        if e is None:
            break
        lr, best = None, None
        for r in range(7):
            if A[r][e] > 0:
                ratio = A[r][nv] / A[r][e]
                if lr is None or ratio < best or (ratio == best and basis[r] < basis[lr]):
                    lr, best = r, ratio
        pv = A[lr][e]
        A[lr] = [a / pv for a in A[lr]]
        for r in range(7):
            if r != lr and A[r][e] != 0:
                f = A[r][e]
                A[r] = [a - f * b for a, b in zip(A[r], A[lr])]
        basis[lr] = e
    return float(sum(A[r][nv] for r in range(7) if basis[r] >= n))


def test_lp_matches_exact_rational_optimum():
    """t* equals the exact rational optimum to 1e-12 on drawn sphere sets
    (long degenerate pivot runs included)."""
    w = synth.workload("c1", n_poses=64)
    fld = oracle.build_field(w.hand, w.field, flags=False)
    Q = oracle.query(w.hand, w.field, fld["bits"], w.obj.pts, w.obj.nrm, w.poses, flags=False)
    spt, _ = oracle.draw(w.hand, w.field, fld["bits"], w.obj.pts, w.obj.nrm, w.poses, Q["dom_bits"],
                         Q["dom_count"], w.search)
    sets = spt.reshape(-1, 3)
    sets = sets[sets[:, 0] >= 0][:24]
    assert len(sets) >= 10
    mu, rho = float(np.float32(0.5)), float(np.float32(w.search.moment_scale))
    for s in sets:
        W = oracle.wrench_matrix(w.obj.pts[s].astype(np.float64), w.obj.nrm[s].astype(np.float64), mu, 8, rho)
        t, st, _ = oracle.lp_solve(W)
        assert st == 0 and abs(t - _exact_tstar(W)) < 1e-12
