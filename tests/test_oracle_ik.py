"""Pins of the oracle's kinematics optimisation (Sec. 5.5, Eq. 7-8, Phase I
and II) against things other than the oracle itself:

* the hand contact point (the capsule point closest to the target in the
  combined position/normal metric) against a dense brute-force minimum over
  the capsule surface refined by a generic optimiser, cylinder, both caps and
  near-ties between them;
* one damped least-squares step at the configured damping against a NumPy
  least-squares solve of the stacked system [J; sqrt(lambda) I] dq = [e; 0],
  with the Jacobian taken by central differences of the forward kinematics;
* the Phase I / Phase II switch: every iteration recomputed from the previous
  iterate, with the contact point held fixed to the link for exactly the
  first ``phase1`` iterations and re-chosen afterwards;
* the witness of the reverse lookup: the smallest joint-sample index reaching
  a (link, voxel, bin) cell, against a brute-force enumeration of every
  contact vector; and the joint sample it names reaches the looked-up cell.
CPU only."""
import math

import numpy as np
import pytest
from scipy.optimize import minimize
from scipy.spatial import cKDTree

import oracle
import synth
from tests.test_oracle_kinematics import planar_2r_hand

BETA = float(np.float32(0.01))


# ---------------------------------------------------------------------------
# hand contact point on a capsule
# ---------------------------------------------------------------------------
def _frame(ax):
    u = np.cross(ax, [1.0, 0.0, 0.0] if abs(ax[0]) < 0.9 else [0.0, 1.0, 0.0])
    u /= np.linalg.norm(u)
    return u, np.cross(ax, u)


def _surface(a, b, r, s_frac, phi, theta, patch):
    """Capsule surface point and outward normal. patch 0: cylinder at axial
    fraction s_frac and angle phi; patch 1 / 2: cap at b / a at polar angle
    theta from the outward axis and azimuth phi."""
    ab = b - a
    L = np.linalg.norm(ab)
    ax = ab / L
    u, w = _frame(ax)
    if patch == 0:
        nu = np.cos(phi) * u + np.sin(phi) * w
        return a + s_frac * ab + r * nu, nu
    sg, c = (1.0, b) if patch == 1 else (-1.0, a)
    nu = np.sin(theta) * (np.cos(phi) * u + np.sin(phi) * w) + sg * np.cos(theta) * ax
    return c + r * nu, nu


def _cost(x, nu, p, n, beta):
    return float(np.sum((x - p) ** 2) + beta * beta * np.sum((nu - n) ** 2))


def _patch_points(a, b, r, patch, s, phi, theta):
    """Vectorised surface points and normals of one patch (arrays of parameters)."""
    ab = b - a
    ax = ab / np.linalg.norm(ab)
    u, w = _frame(ax)
    radial = np.cos(phi)[:, None] * u + np.sin(phi)[:, None] * w
    if patch == 0:
        nu = radial
        return a + s[:, None] * ab + r * nu, nu
    sg, c = (1.0, b) if patch == 1 else (-1.0, a)
    nu = np.sin(theta)[:, None] * radial + sg * np.cos(theta)[:, None] * ax
    return c + r * nu, nu


def _brute_min(a, b, r, p, n, beta):
    """Dense sampling of the three patches, then Nelder-Mead from the best
    sample of each patch (parameters clamped into the patch)."""
    best = (math.inf, None, None, None)
    S, PH = np.meshgrid(np.linspace(0.0, 1.0, 121), np.linspace(0.0, 2 * np.pi, 181, endpoint=False), indexing="ij")
    TH, PH2 = np.meshgrid(np.linspace(0.0, np.pi / 2, 61), np.linspace(0.0, 2 * np.pi, 181, endpoint=False),
                          indexing="ij")
    for patch in range(3):
        if patch == 0:
            s, ph, th = S.ravel(), PH.ravel(), np.zeros(S.size)
        else:
            s, ph, th = np.zeros(TH.size), PH2.ravel(), TH.ravel()
        x, nu = _patch_points(a, b, r, patch, s, ph, th)
        costs = ((x - p) ** 2).sum(1) + beta * beta * ((nu - n) ** 2).sum(1)
        i0 = int(np.argmin(costs))

        def obj(v, patch=patch):
            if patch == 0:
                x, nu = _surface(a, b, r, min(max(v[0], 0.0), 1.0), v[1], 0.0, 0)
            else:
                x, nu = _surface(a, b, r, 0.0, v[1], min(max(v[0], 0.0), np.pi / 2), patch)
            return _cost(x, nu, p, n, beta)
        v0 = [s[i0], ph[i0]] if patch == 0 else [th[i0], ph[i0]]
        res = minimize(obj, v0, method="Nelder-Mead", options={"xatol": 1e-12, "fatol": 1e-18, "maxiter": 4000})
        if res.fun < best[0]:
            v = res.x
            if patch == 0:
                x, nu = _surface(a, b, r, min(max(v[0], 0.0), 1.0), v[1], 0.0, 0)
            else:
                x, nu = _surface(a, b, r, 0.0, v[1], min(max(v[0], 0.0), np.pi / 2), patch)
            best = (res.fun, x, nu, patch)
    return best


def _on_capsule(a, b, r, x, nu):
    ab = b - a
    t = np.clip(np.dot(x - a, ab) / np.dot(ab, ab), 0.0, 1.0)
    c = a + t * ab
    return abs(np.linalg.norm(x - c) - r) < 1e-12 and np.allclose((x - c) / r, nu, atol=1e-10)


def test_capsule_contact_point_is_the_brute_force_minimum():
    """The chosen point lies on the capsule with its outward normal and its
    cost is the surface minimum (a point of the dense sampling refined by a
    generic optimiser is never better); where the minimum is clear the two
    points coincide.  Targets all around the capsule reach the cylinder and
    both caps."""
    rng = np.random.default_rng(21)
    patches = set()
    for trial in range(60):
        a = rng.normal(0, 0.02, 3)
        ax = rng.normal(size=3)
        ax /= np.linalg.norm(ax)
        L, r = rng.uniform(0.02, 0.05), rng.uniform(0.006, 0.01)
        b = a + L * ax
        # target: around the capsule, from inside it to 2 cm out, any side
        t = rng.uniform(-0.4, 1.4)
        off = rng.normal(size=3)
        off -= np.dot(off, ax) * ax
        off /= np.linalg.norm(off)
        p = a + t * (b - a) + rng.uniform(0.0, r + 0.02) * off
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        got = oracle.capsule_aligned_point(a, b, r, p, n, BETA)
        assert _on_capsule(a, b, r, got["pt"], got["nt"])
        c_o = _cost(got["pt"], got["nt"], p, n, BETA)
        c_b, xb, nub, patch = _brute_min(a, b, r, p, n, BETA)
        patches.add(patch)
        assert c_o <= c_b + 1e-14, (trial, c_o, c_b)
        if got["gap"] > 1e-4:
            assert np.linalg.norm(got["pt"] - xb) < 1e-5, trial
    assert patches == {0, 1, 2}


def test_capsule_contact_point_near_ties_and_their_margin():
    """A target on the capsule axis beyond the end cap with a normal tilted off
    the axis: the cap and the cylinder rim compete.  Sliding the target along
    the axis moves the minimum from one to the other; the oracle follows the
    brute-force winner on both sides and reports a tie margin that shrinks to
    zero at the crossing."""
    a, b, r = np.zeros(3), np.array([0.0, 0.0, 0.03]), 0.008
    n = np.array([math.sin(1.2), 0.0, math.cos(1.2)])
    # inside the capsule near the end cap centre: cap pulls towards +z, cylinder sideways
    zs = np.linspace(0.015, 0.034, 60)
    which = []
    for z in zs:
        p = np.array([0.0, 0.0, z])
        got = oracle.capsule_aligned_point(a, b, r, p, n, BETA)
        on_cap = got["pt"][2] > b[2] + 1e-9 or np.dot(got["nt"], [0, 0, 1.0]) > 1e-9
        which.append(on_cap)
        c_b, xb, nub, patch = _brute_min(a, b, r, p, n, BETA)
        c_o = _cost(got["pt"], got["nt"], p, n, BETA)
        assert c_o <= c_b + 1e-14
    which = np.array(which)
    assert which.any() and (~which).any(), "no crossing between cylinder and cap on this path"
    # locate the crossing by bisection and check the reported margin there
    i = int(np.flatnonzero(which != which[0])[0])
    lo, hi = zs[i - 1], zs[i]
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        g = oracle.capsule_aligned_point(a, b, r, np.array([0, 0, mid]), n, BETA)
        m_cap = g["pt"][2] > b[2] + 1e-9 or np.dot(g["nt"], [0, 0, 1.0]) > 1e-9
        if m_cap == which[0]:
            lo = mid
        else:
            hi = mid
    g_tie = oracle.capsule_aligned_point(a, b, r, np.array([0, 0, lo]), n, BETA)
    g_far = oracle.capsule_aligned_point(a, b, r, np.array([0, 0, zs[0]]), n, BETA)
    assert g_tie["gap"] < 1e-9 < g_far["gap"]


# ---------------------------------------------------------------------------
# one damped least-squares step, and the Phase I / II switch
# ---------------------------------------------------------------------------
def _link_point_fn(hand, f, l, q_full, local):
    js = hand.finger_joints(f)

    def x_of(qf):
        q = q_full.copy()
        q[js] = qf
        T = oracle.fk(hand, q)[l].reshape(3, 4)
        return T[:, :3] @ local + T[:, 3]
    return x_of


def _cd_jacobian(fn, q, h=1e-6):
    cols = []
    for t in range(len(q)):
        dq = np.zeros(len(q))
        dq[t] = h
        cols.append((fn(q + dq) - fn(q - dq)) / (2 * h))
    return np.stack(cols, axis=1)


def _select(hand, f, l, qf, p, n, beta):
    """Contact point chosen at finger configuration qf: world point, normal and
    their link-frame coordinates."""
    js = hand.finger_joints(f)
    q = np.zeros(hand.n_joints)
    q[js] = qf
    T = oracle.fk(hand, q)[l].reshape(3, 4)
    cap = hand.capsule[l].astype(np.float64)
    A, B = T[:, :3] @ cap[:3] + T[:, 3], T[:, :3] @ cap[3:6] + T[:, 3]
    got = oracle.capsule_aligned_point(A, B, float(cap[6]), p, n, beta)
    loc_p = T[:, :3].T @ (got["pt"] - T[:, 3])
    loc_n = T[:, :3].T @ got["nt"]
    return loc_p, loc_n


def _dls_step(hand, f, l, qf, p, n, loc_p, loc_n, lam, beta):
    """q' = clip(q + dq), dq the least-squares solution of
    [J; sqrt(lam) I] dq = [e; 0] (numerically: SVD), J by central differences."""
    js = hand.finger_joints(f)
    qfull = np.zeros(hand.n_joints)
    x1 = _link_point_fn(hand, f, l, qfull, loc_p)
    x2 = _link_point_fn(hand, f, l, qfull, loc_p + beta * loc_n)
    e = np.concatenate([p - x1(qf), (p + beta * n) - x2(qf)])
    Jm = np.vstack([_cd_jacobian(x1, qf), _cd_jacobian(x2, qf)])
    d = len(qf)
    A = np.vstack([Jm, math.sqrt(lam) * np.eye(d)])
    rhs = np.concatenate([e, np.zeros(d)])
    dq = np.linalg.lstsq(A, rhs, rcond=None)[0]
    lo, hi = hand.limits[js, 0].astype(np.float64), hand.limits[js, 1].astype(np.float64)
    return np.clip(qf + dq, lo, hi)


def _target(hand, f, l, rng):
    """A contact target near (not on) link l: a point of the link surface at a
    random interior configuration, displaced by a few millimetres, with a
    tilted normal."""
    js = hand.finger_joints(f)
    lo, hi = hand.limits[js, 0].astype(np.float64), hand.limits[js, 1].astype(np.float64)
    qs = rng.uniform(lo + 0.25 * (hi - lo), hi - 0.25 * (hi - lo))
    q = np.zeros(hand.n_joints)
    q[js] = qs
    T = oracle.fk(hand, q)[l].reshape(3, 4)
    cap = hand.capsule[l].astype(np.float64)
    ph = rng.uniform(0, 2 * np.pi)
    nl = np.array([math.cos(ph), math.sin(ph), 0.0])
    loc = cap[:3] + rng.uniform(0.2, 0.9) * (cap[3:6] - cap[:3]) + cap[6] * nl
    p = T[:, :3] @ loc + T[:, 3] + rng.normal(0, 0.004, 3)
    n = T[:, :3] @ nl + rng.normal(0, 0.2, 3)
    n /= np.linalg.norm(n)
    q0 = np.clip(qs + rng.normal(0, 0.15, len(js)), lo + 1e-3, hi - 1e-3)
    return p, n, q0


def test_one_dls_step_at_configured_damping_matches_stacked_least_squares():
    """One iteration of the oracle's IK at lambda = 1e-2 equals the
    least-squares step of [J; sqrt(lambda) I] dq = [e; 0] (Eq. 7, damped),
    J by central differences of the FK of the contact point and of the point
    beta along its normal, both fixed to the link (Eq. 8)."""
    hand = synth.hand_c3()
    ik = synth.IKParams(iters=1)
    lam = float(np.float32(ik.lam))
    rng = np.random.default_rng(31)
    n_checked = 0
    for trial in range(40):
        f = int(rng.integers(0, hand.n_fingers))
        js = hand.finger_joints(f)
        l = int(js[rng.integers(1, len(js))])
        p, n, q0 = _target(hand, f, l, rng)
        out = oracle.ik_finger(hand, f, l, p, n, q0, ik)
        loc_p, loc_n = _select(hand, f, l, q0, p, n, BETA)
        want = _dls_step(hand, f, l, q0, p, n, loc_p, loc_n, lam, BETA)
        assert np.abs(out["q"] - want).max() < 1e-8, (trial, out["q"] - want)
        # the damping is what the check sees: lambda^2 would move q visibly
        alt = _dls_step(hand, f, l, q0, p, n, loc_p, loc_n, lam * lam, BETA)
        n_checked += np.abs(alt - want).max() > 1e-5
    assert n_checked >= 30


def test_phase_one_holds_the_link_point_for_exactly_phase1_iterations():
    """Each iterate q_{i+1} is one damped step from q_i: for i < phase1 with the
    contact point chosen at q_0 and carried on the link, for i >= phase1 with
    the point chosen again at q_i.  The cases are built so that the two rules
    give visibly different steps at i = phase1 (an off-by-one switch fails)."""
    hand = synth.hand_c3()
    lam = float(np.float32(1e-2))
    rng = np.random.default_rng(41)
    discriminating = 0
    for trial in range(12):
        f = int(rng.integers(0, hand.n_fingers))
        js = hand.finger_joints(f)
        l = int(js[-1])
        p, n, q0 = _target(hand, f, l, rng)
        ik_full = synth.IKParams()
        P1 = ik_full.phase1
        qs = [q0]
        for i in range(1, ik_full.iters + 1):
            qs.append(oracle.ik_finger(hand, f, l, p, n, q0, synth.IKParams(iters=i))["q"])
        loc0 = _select(hand, f, l, q0, p, n, BETA)
        for i in range(ik_full.iters):
            fixed = _dls_step(hand, f, l, qs[i], p, n, *loc0, lam, BETA)
            again = _dls_step(hand, f, l, qs[i], p, n, *_select(hand, f, l, qs[i], p, n, BETA), lam, BETA)
            want = fixed if i < P1 else again
            assert np.abs(qs[i + 1] - want).max() < 1e-8, (trial, i)
            if i == P1:
                discriminating += np.abs(fixed - again).max() > 1e-6
        # the last iterate is the full run's result
        assert np.abs(oracle.ik_finger(hand, f, l, p, n, q0, ik_full)["q"] - qs[-1]).max() == 0.0
    assert discriminating >= 6


# ---------------------------------------------------------------------------
# witness of the reverse lookup
# ---------------------------------------------------------------------------
def test_witness_is_the_smallest_reaching_sample():
    """Every field cell's witness is the smallest joint-sample index of a
    contact vector landing in it, from an enumeration of all (sample, link,
    surface sample) vectors with a KD-tree bin search; cells that a vector
    reaches within 1e-6 m of a voxel face or 1e-6 rad of a bin boundary are
    left out (either neighbour is correct there)."""
    h = planar_2r_hand(tip_only=False)
    G, hv, B, S = 16, 0.008, 32, 96
    Rw = np.eye(3)
    centre = np.array([0.0013, -0.045, 0.025])
    gf = np.zeros((1, 12), np.float32)
    gf[0] = synth._pack34(Rw, centre - np.full(3, 0.5 * G * hv))
    fp = synth.FieldParams(samples=S, seed=3, grid=G, h=hv, bins=B, grid_frame=gf)
    fld = oracle.build_field(h, fp, witness=True, flags=False)
    wit = fld["wit"]
    c = oracle.bin_centers(B)
    tree = cKDTree(c)
    og = gf[0].reshape(3, 4)[:, 3].astype(np.float64)
    hh = float(np.float32(hv))
    want = np.full(wit.shape, -1, np.int64)
    risky = np.zeros(wit.shape, bool)
    for s in range(S):
        q = np.zeros(h.n_joints)
        q[h.finger_joints(0)] = oracle.joint_sample(h, fp.seed, 0, s)
        T = oracle.fk(h, q)
        for l in range(h.n_joints):
            Tl = T[l].reshape(3, 4)
            sp = h.surf[l].astype(np.float64)
            x = sp[:, :3] @ Tl[:, :3].T + Tl[:, 3]
            nu = sp[:, 3:] @ Tl[:, :3].T
            nu /= np.linalg.norm(nu, axis=1, keepdims=True)
            u = (x - og) / hh
            ins = np.all((u >= 0) & (u < G), axis=1)
            dd, bb = tree.query(nu, k=2)
            ang = np.arccos(np.clip(nu @ c.T, -1, 1))
            gap = 0.5 * (np.take_along_axis(ang, bb[:, 1:2], 1) - np.take_along_axis(ang, bb[:, :1], 1))[:, 0]
            fr = u - np.floor(u)
            near = (np.minimum(fr, 1 - fr).min(axis=1) * hh < 1e-6) | (gap < 1e-6)
            for i in np.flatnonzero(ins):
                v = (int(u[i, 2]) * G + int(u[i, 1])) * G + int(u[i, 0])
                cell = (l, v, int(bb[i, 0]))
                if want[cell] < 0 or s < want[cell]:
                    want[cell] = s
                risky[cell] |= near[i]
    assert (want >= 0).sum() > 100
    ok = ~risky
    assert np.array_equal(wit[ok], want[ok])


def test_reverse_lookup_witness_reaches_the_contact_cell():
    """For realised contacts the starting configuration q0 is the witness
    sample of the looked-up (link, voxel(p), bin(n)) cell: some surface sample
    of that link, at q0, lands in the same voxel and bin as the contact
    (recomputed here with the window frame and a KD-tree bin search), unless
    the lookup is flagged."""
    w = synth.workload("c1", with_sdf=True)
    ref = oracle.build_field(w.hand, w.field, witness=True, flags=False)
    Q = oracle.query(w.hand, w.field, ref["bits"], w.obj.pts, w.obj.nrm, w.poses, flags=False)
    spt, sln = oracle.draw(w.hand, w.field, ref["bits"], w.obj.pts, w.obj.nrm, w.poses, Q["dom_bits"],
                           Q["dom_count"], w.search)
    V = oracle.verdicts(w.obj.pts, w.obj.nrm, spt, w.search)
    acc = oracle.compact(V["verdict"])[:400]
    k = w.search.k
    R = oracle.realize(w.hand, w.field, ref["wit"], w.sdf, w.obj.pts, w.obj.nrm, w.poses, spt.reshape(-1, k),
                       sln.reshape(-1, k), w.search, acc, w.ik)
    tree = cKDTree(oracle.bin_centers(w.field.bins))
    G, hh = w.field.grid, float(np.float32(w.field.h))
    checked = 0
    for a, sid in enumerate(acc):
        if R["rflag"][a] & 2:
            continue
        g = sid // w.search.draws
        P = w.poses[g].reshape(3, 4).astype(np.float64)
        T0 = oracle.fk(w.hand, R["q0"][a])
        for i in range(k):
            idx, l = int(spt.reshape(-1, k)[sid, i]), int(sln.reshape(-1, k)[sid, i])
            f = int(w.hand.joint_finger[l])
            p = P[:, :3] @ w.obj.pts[idx].astype(np.float64) + P[:, 3]
            n = -(P[:, :3] @ w.obj.nrm[idx].astype(np.float64))
            Fw = w.field.grid_frame[f].reshape(3, 4).astype(np.float64)
            vox = np.floor(Fw[:, :3].T @ (p - Fw[:, 3]) / hh).astype(int)
            b = tree.query(n / np.linalg.norm(n))[1]
            Tl = T0[l].reshape(3, 4)
            sp = w.hand.surf[l].astype(np.float64)
            x = sp[:, :3] @ Tl[:, :3].T + Tl[:, 3]
            nu = sp[:, 3:] @ Tl[:, :3].T
            vs = np.floor((x - Fw[:, 3]) @ Fw[:, :3] / hh).astype(int)
            bs = tree.query(nu / np.linalg.norm(nu, axis=1, keepdims=True))[1]
            hit = np.all(vs == vox, axis=1) & (bs == b)
            assert hit.any(), (a, i)
            checked += 1
    assert checked > 150
