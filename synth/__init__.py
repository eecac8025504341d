"""Seeded synthetic inputs: hands, objects, palm poses and object SDF grids.

This module only builds *inputs*.  It holds none of the method's arithmetic:
no forward kinematics, no field binning, no contact-domain query, no draws,
no force-closure LP, no IK and no penetration test.  Both the FP64 CPU oracle
(``oracle/``) and the HIP library (``paper_2511_07418_amd/``) consume exactly
the float32 arrays produced here, so parity tests compare the two on identical
inputs.

All geometry is generated in float64 with NumPy's PCG64 generator (seeded
through ``SeedSequence([seed, tag])``) and emitted as float32.  Units are SI
(metres, radians).

Workload recipes (the paper's hands and objects -- Allegro/LEAP/Shadow/DClaw,
YCB and Sketchfab meshes, Sec. 6 and Table 1 -- are not available; these
stand-ins keep their shape: 9/16/22-DOF multi-finger hands and regular,
superquadric and tool-like objects):

* ``c1`` tiny   : 3 fingers x 3 flexion joints (9 DOF), sphere R=40 mm,
                  N=2,048, P=256, D=16, k=3, field 32^3 @ 4 mm, 32 bins,
                  S=8,192 joint samples per finger.
* ``c2`` mid    : 4 fingers x 4 joints (16 DOF), superquadric, N=16,384,
                  P=16,384, D=32, k=4, field 64^3 @ 3 mm, 64 bins, S=262,144.
* ``c3`` full   : 5 fingers, 22 DOF, tool-like union of 2-6 ellipsoids and
                  capsules, N=65,536, P=65,536, D=64, k=5, field as c2,
                  IK 10 iterations (lambda=1e-2), SDF 64^3.

Each workload function accepts overrides (``n_points``, ``n_poses``,
``samples``...) so tests can keep the exact shapes of a config while shrinking
the parts the CPU oracle must enumerate.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

GOLDEN = math.pi * (3.0 - math.sqrt(5.0))  # golden angle (rad)

# seed-sequence tags, one per generator purpose
_TAG_HAND, _TAG_OBJ, _TAG_POSE, _TAG_SDF = 101, 102, 103, 104


def _rng(seed: int, tag: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([int(seed), int(tag)]))


# --------------------------------------------------------------------------
# small rigid-transform helpers (input construction only)
# --------------------------------------------------------------------------
def _pack34(R: np.ndarray, t: np.ndarray) -> np.ndarray:
    """3x4 row-major [R | t] flattened to 12 numbers."""
    M = np.zeros((3, 4))
    M[:, :3] = R
    M[:, 3] = t
    return M.reshape(12)


def _finger_base_rotation(phi: float, splay: float = 0.0) -> np.ndarray:
    """Base frame of a finger standing on the palm at azimuth ``phi``.

    Columns before splay: x = tangent (flexion axis), y = radial outward,
    z = palm normal.  A positive rotation about x turns the link direction
    (+z) towards -y, i.e. the finger curls towards the palm centre.  ``splay``
    tilts the rest direction outwards (rotation by -splay about x), so the
    open hand is a claw that closes by flexion.
    """
    x = np.array([math.sin(phi), -math.cos(phi), 0.0])
    y = np.array([math.cos(phi), math.sin(phi), 0.0])
    z = np.array([0.0, 0.0, 1.0])
    R = np.stack([x, y, z], axis=1)
    c, s = math.cos(-splay), math.sin(-splay)
    Rx = np.array([[1.0, 0.0, 0.0], [0.0, c, -s], [0.0, s, c]])
    return R @ Rx


# --------------------------------------------------------------------------
# hands
# --------------------------------------------------------------------------
@dataclass
class Hand:
    """Capsule-chain hand: one link (capsule) per revolute joint.

    Joints are grouped by finger (a finger is one dependency group, Sec. 5.3);
    within a finger they form a serial chain in array order.  Frame of joint j:
    ``T_j = T_parent * origin_j * Rot(axis_j, q_j)`` with ``T_parent`` the hand
    base frame for the first joint of a finger.
    """
    n_fingers: int
    joint_finger: np.ndarray   # int32 [J]
    joint_parent: np.ndarray   # int32 [J]  (-1: attached to the hand base)
    joint_origin: np.ndarray   # float32 [J,12] parent->joint 3x4 at q=0
    joint_axis: np.ndarray     # float32 [J,3] unit axis in the joint frame
    capsule: np.ndarray        # float32 [J,7] a(3), b(3), radius in link frame
    limits: np.ndarray         # float32 [J,2] lo, hi
    surf: np.ndarray           # float32 [J,S_p,6] link-frame point, outward normal
    finger_base: np.ndarray    # float64 [F,3,4] base frame of each finger (for grid placement)

    @property
    def n_joints(self) -> int:
        return int(self.joint_finger.shape[0])

    def finger_joints(self, f: int) -> np.ndarray:
        return np.nonzero(self.joint_finger == f)[0]

    @property
    def dof(self) -> list[int]:
        return [int((self.joint_finger == f).sum()) for f in range(self.n_fingers)]


def capsule_surface_samples(length: float, radius: float, n: int) -> np.ndarray:
    """Area-uniform deterministic samples of a capsule along +z from 0 to ``length``.

    The count is split by area between the cylinder (golden-angle lattice on
    evenly spaced rings) and the two hemispherical caps (Fibonacci caps).
    Returns float64 [n, 6]: point, outward unit normal.
    """
    a_cyl = 2.0 * math.pi * radius * length
    a_cap = 2.0 * math.pi * radius * radius  # one hemisphere
    n_cyl = int(round(n * a_cyl / (a_cyl + 2.0 * a_cap)))
    n_caps = n - n_cyl
    n_top = (n_caps + 1) // 2
    n_bot = n_caps - n_top
    out = []
    for i in range(n_cyl):
        z = (i + 0.5) / n_cyl * length
        ph = i * GOLDEN
        c, s = math.cos(ph), math.sin(ph)
        out.append((radius * c, radius * s, z, c, s, 0.0))
    for (cnt, zc, sgn) in ((n_top, length, 1.0), (n_bot, 0.0, -1.0)):
        for i in range(cnt):
            cz = 1.0 - (i + 0.5) / cnt  # cos(polar) in (0, 1]
            sz = math.sqrt(max(0.0, 1.0 - cz * cz))
            ph = i * GOLDEN
            d = (sz * math.cos(ph), sz * math.sin(ph), sgn * cz)
            out.append((radius * d[0], radius * d[1], zc + radius * d[2], d[0], d[1], d[2]))
    return np.asarray(out, dtype=np.float64)


def _build_hand(fingers: list[dict], n_surf: int) -> Hand:
    """fingers: list of {base: (R, t), joints: [(axis_local, length, radius, lo, hi)]}."""
    jf, jp, jo, ja, cap, lim, surf, bases = [], [], [], [], [], [], [], []
    j = 0
    for f, fd in enumerate(fingers):
        R0, t0 = fd["base"]
        bases.append(np.concatenate([R0, t0[:, None]], axis=1))
        prev_len = None
        for (axis, length, radius, lo, hi) in fd["joints"]:
            jf.append(f)
            if prev_len is None:
                jp.append(-1)
                jo.append(_pack34(R0, t0))
            else:
                jp.append(j - 1)
                jo.append(_pack34(np.eye(3), np.array([0.0, 0.0, prev_len])))
            ja.append(np.asarray(axis, dtype=np.float64))
            cap.append(np.array([0.0, 0.0, 0.0, 0.0, 0.0, length, radius]))
            lim.append(np.array([lo, hi]))
            surf.append(capsule_surface_samples(length, radius, n_surf))
            prev_len = length
            j += 1
    return Hand(
        n_fingers=len(fingers),
        joint_finger=np.asarray(jf, np.int32),
        joint_parent=np.asarray(jp, np.int32),
        joint_origin=np.asarray(jo, np.float64).astype(np.float32),
        joint_axis=np.asarray(ja, np.float64).astype(np.float32),
        capsule=np.asarray(cap, np.float64).astype(np.float32),
        limits=np.asarray(lim, np.float64).astype(np.float32),
        surf=np.asarray(surf, np.float64).astype(np.float32),
        finger_base=np.asarray(bases, np.float64),
    )


X_AX, Y_AX, Z_AX = (1.0, 0.0, 0.0), (0.0, 1.0, 0.0), (0.0, 0.0, 1.0)


def hand_c1(n_surf: int = 256, splay: float = 0.9) -> Hand:
    """3 planar-base fingers x 3 flexion joints (9 DOF); capsules r=8 mm,
    lengths 45/30/25 mm, limits [0, 1.6] rad, bases at 0/120/240 deg on a
    30 mm circle."""
    fingers = []
    for phi_deg in (0.0, 120.0, 240.0):
        phi = math.radians(phi_deg)
        R0 = _finger_base_rotation(phi, splay)
        t0 = np.array([0.03 * math.cos(phi), 0.03 * math.sin(phi), 0.0])
        fingers.append({"base": (R0, t0), "joints": [
            (X_AX, L, 0.008, 0.0, 1.6) for L in (0.045, 0.030, 0.025)]})
    return _build_hand(fingers, n_surf)


def hand_c2(seed: int = 0, n_surf: int = 256, splay: float = 0.9) -> Hand:
    """4 fingers x 4 joints (16 DOF): joint 0 abduction (radial axis), joints
    1-3 flexion; r=9 mm, lengths U[20,50] mm, limits [-0.3, 1.7] rad."""
    rng = _rng(seed, _TAG_HAND)
    lengths = rng.uniform(0.020, 0.050, size=(4, 4))
    fingers = []
    for f, phi_deg in enumerate((0.0, 90.0, 180.0, 270.0)):
        phi = math.radians(phi_deg)
        R0 = _finger_base_rotation(phi, splay)
        t0 = np.array([0.03 * math.cos(phi), 0.03 * math.sin(phi), 0.0])
        joints = [(Y_AX, lengths[f, 0], 0.009, -0.3, 1.7)]
        joints += [(X_AX, lengths[f, i], 0.009, -0.3, 1.7) for i in (1, 2, 3)]
        fingers.append({"base": (R0, t0), "joints": joints})
    return _build_hand(fingers, n_surf)


def hand_c3(seed: int = 0, n_surf: int = 256, splay: float = 0.9) -> Hand:
    """5 fingers, 22 DOF.  Thumb (5): abduction, twist, 3 flexion.  Index,
    middle, ring (4 each): abduction + 3 flexion.  Little (5): a palm
    (metacarpal) flexion joint, abduction, 3 flexion.  r=9 mm, lengths
    U[20,50] mm."""
    rng = _rng(seed, _TAG_HAND)
    r = 0.009
    flex = (-0.3, 1.7)
    spec = [
        # (azimuth deg, base radius, joints [(axis, lo, hi)])
        (180.0, 0.035, [(Y_AX, -0.5, 0.5), (Z_AX, -0.8, 0.8)] + [(X_AX, *flex)] * 3),
        (60.0, 0.040, [(Y_AX, -0.4, 0.4)] + [(X_AX, *flex)] * 3),
        (20.0, 0.040, [(Y_AX, -0.4, 0.4)] + [(X_AX, *flex)] * 3),
        (-20.0, 0.040, [(Y_AX, -0.4, 0.4)] + [(X_AX, *flex)] * 3),
        (-60.0, 0.040, [(X_AX, 0.0, 0.8), (Y_AX, -0.4, 0.4)] + [(X_AX, *flex)] * 3),
    ]
    fingers = []
    for (phi_deg, rad, joints) in spec:
        phi = math.radians(phi_deg)
        R0 = _finger_base_rotation(phi, splay)
        t0 = np.array([rad * math.cos(phi), rad * math.sin(phi), 0.0])
        lens = rng.uniform(0.020, 0.050, size=len(joints))
        fingers.append({"base": (R0, t0), "joints": [
            (ax, float(L), r, lo, hi) for (ax, lo, hi), L in zip(joints, lens)]})
    return _build_hand(fingers, n_surf)


@dataclass
class Palm:
    """Static link of the hand (the palm, Sec. 5.1 static-link contacts): a
    disc of radius R at z = 0 of the hand base frame, facing +z.

    surf: float32 [S,6] contact vectors (point on the disc, normal +z), a
    Fibonacci disc lattice; caps: float32 [C,7] capsules a(3), b(3), radius in
    the base frame -- parallel rods of radius r_c along x at z = -r_c whose
    tops reach the disc plane, at most 1.6 r_c apart in y, each as long as the
    disc's chord at its y."""
    surf: np.ndarray
    caps: np.ndarray
    radius: float


def palm_disc(radius: float, n_surf: int = 512, rod: float = 0.005) -> Palm:
    i = np.arange(n_surf) + 0.5
    r = radius * np.sqrt(i / n_surf)
    ph = np.arange(n_surf) * GOLDEN
    surf = np.zeros((n_surf, 6))
    surf[:, 0], surf[:, 1], surf[:, 5] = r * np.cos(ph), r * np.sin(ph), 1.0
    caps = []
    edge = radius - 0.8 * rod
    n_rods = int(math.floor(2 * edge / (1.6 * rod))) + 1
    for y in np.linspace(-edge, edge, n_rods):
        hx = math.sqrt(radius * radius - y * y)
        caps.append((-hx, y, -rod, hx, y, -rod, rod))
    return Palm(surf=surf.astype(np.float32), caps=np.asarray(caps, np.float32), radius=radius)


def palm_for(name: str) -> Palm:
    """The palm of workload ``name``'s hand: inside the circle of finger bases
    (30 mm for c1/c2, 35-40 mm for c3)."""
    return palm_disc({"c1": 0.025, "c2": 0.025, "c3": 0.030}[name])


# --------------------------------------------------------------------------
# contact-field grid placement
# --------------------------------------------------------------------------
@dataclass
class FieldParams:
    samples: int               # S joint samples per finger
    seed: int                  # Philox key (64 bit)
    grid: int                  # G (G^3 voxels per finger window)
    h: float                   # voxel edge (m)
    bins: int                  # B normal bins (32 or 64)
    grid_frame: np.ndarray     # float32 [F,12]: 3x4 [R | o]; voxel coords u = R^T (x - o) / h


# Grid centre of a finger window, in the finger base frame, as a fraction of
# the finger's reach (total link length + radius).  Flexion curls towards -y,
# so the reachable set lies mostly on the palm side (-y) and above the palm.
GRID_CENTER_FRAC = (0.0, -0.30, 0.22)
# Shift of the window lattice off the hand frame's planes (voxel units), so
# that symmetry planes of the hand (a planar finger's flexion plane through a
# base axis) do not coincide with voxel faces.
GRID_LATTICE_SHIFT = (0.37, 0.29, 0.41)
# Window origins sit on a lattice of this many voxels (the field's brick edge).
GRID_SNAP = 4


def grid_frames(hand: Hand, G: int, h: float) -> np.ndarray:
    """Per-finger grid frames, all with the axes of the hand (palm) frame.
    Finger f's G^3 window is centred near a fixed fraction of the finger's
    reach, placed along the finger's base frame; its origin is snapped to a
    lattice of GRID_SNAP voxels shifted by GRID_LATTICE_SHIFT, shared by all
    fingers, so the windows differ by whole bricks.  No kinematics is
    evaluated; only link lengths enter."""
    out = []
    shift = np.array(GRID_LATTICE_SHIFT) * h
    for f in range(hand.n_fingers):
        js = hand.finger_joints(f)
        reach = float(hand.capsule[js, 5].astype(np.float64).sum() + hand.capsule[js[0], 6])
        Rb = hand.finger_base[f][:, :3].astype(np.float64)
        tb = hand.finger_base[f][:, 3].astype(np.float64)
        centre = tb + Rb @ (np.array(GRID_CENTER_FRAC) * reach)
        step = GRID_SNAP * h
        o = np.round((centre - 0.5 * G * h - shift) / step) * step + shift
        out.append(_pack34(np.eye(3), o))
    return np.asarray(out, np.float64).astype(np.float32)


def grid_frames_finger_aligned(hand: Hand, G: int, h: float) -> np.ndarray:
    """Per-finger grid frames with the axes of each finger's base frame (no
    shared rotation, no common lattice): windows mapped finger by finger."""
    out = []
    for f in range(hand.n_fingers):
        js = hand.finger_joints(f)
        reach = float(hand.capsule[js, 5].astype(np.float64).sum() + hand.capsule[js[0], 6])
        Rb = hand.finger_base[f][:, :3]
        tb = hand.finger_base[f][:, 3]
        c_local = np.array(GRID_CENTER_FRAC) * reach + np.array([GRID_LATTICE_SHIFT[0] * h, 0.0, 0.0])
        o_local = c_local - 0.5 * G * h
        o = tb + Rb @ o_local
        out.append(_pack34(Rb, o))
    return np.asarray(out, np.float64).astype(np.float32)


# --------------------------------------------------------------------------
# objects
# --------------------------------------------------------------------------
@dataclass
class Obj:
    pts: np.ndarray            # float32 [N,3] object frame, Morton-sorted
    nrm: np.ndarray            # float32 [N,3] outward unit normals
    rho: float                 # moment scale: max |p_i|
    kind: str
    params: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.pts.shape[0])

    def soa(self) -> tuple[np.ndarray, np.ndarray]:
        """Structure-of-arrays [3][N] float32 copies (the library layout)."""
        return (np.ascontiguousarray(self.pts.T.astype(np.float32)),
                np.ascontiguousarray(self.nrm.T.astype(np.float32)))


def morton_order(p: np.ndarray, bits: int = 10) -> np.ndarray:
    """Permutation sorting points along a 3-D Morton (Z-order) curve."""
    lo, hi = p.min(axis=0), p.max(axis=0)
    span = np.maximum(hi - lo, 1e-12)
    q = np.clip(((p - lo) / span * ((1 << bits) - 1)).astype(np.int64), 0, (1 << bits) - 1)
    code = np.zeros(p.shape[0], dtype=np.int64)
    for b in range(bits):
        for a in range(3):
            code |= ((q[:, a] >> b) & 1) << (3 * b + a)
    return np.argsort(code, kind="stable")


def _finish_object(p: np.ndarray, n: np.ndarray, kind: str, params: dict) -> Obj:
    n = n / np.linalg.norm(n, axis=1, keepdims=True)
    order = morton_order(p)
    p, n = p[order], n[order]
    rho = float(np.linalg.norm(p.astype(np.float32).astype(np.float64), axis=1).max())
    return Obj(pts=p.astype(np.float32), nrm=n.astype(np.float32), rho=rho, kind=kind, params=params)


def sphere_object(radius: float = 0.04, n: int = 2048) -> Obj:
    """Fibonacci-sampled sphere with outward normals."""
    i = np.arange(n, dtype=np.float64)
    z = 1.0 - (2.0 * i + 1.0) / n
    s = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    ph = i * GOLDEN
    d = np.stack([s * np.cos(ph), s * np.sin(ph), z], axis=1)
    return _finish_object(radius * d, d, "sphere", {"radius": radius})


def _spow(x, e):
    return np.sign(x) * np.abs(x) ** e


def _sq_surface(a, b, c, e1, e2, eta, om):
    ce, se, co, so = np.cos(eta), np.sin(eta), np.cos(om), np.sin(om)
    return np.stack([a * _spow(ce, e1) * _spow(co, e2),
                     b * _spow(ce, e1) * _spow(so, e2),
                     c * _spow(se, e1)], axis=1)


def _sq_area_uniform(rng, a, b, c, e1, e2, n, replace=False):
    """(eta, omega) of n area-uniform superquadric samples: parametric
    oversampling (8n) and area-weighted resampling (without replacement for
    object points; with replacement, which is much faster, for SDF samples)."""
    m = 8 * n
    eta = rng.uniform(-0.5 * math.pi, 0.5 * math.pi, size=m)
    om = rng.uniform(-math.pi, math.pi, size=m)
    d = 1e-6
    pe = (_sq_surface(a, b, c, e1, e2, eta + d, om) - _sq_surface(a, b, c, e1, e2, eta - d, om)) / (2 * d)
    po = (_sq_surface(a, b, c, e1, e2, eta, om + d) - _sq_surface(a, b, c, e1, e2, eta, om - d)) / (2 * d)
    dA = np.linalg.norm(np.cross(pe, po), axis=1)
    dA = np.nan_to_num(dA, nan=0.0, posinf=0.0)
    pick = rng.choice(m, size=n, replace=replace, p=dA / dA.sum())
    return eta[pick], om[pick]


def superquadric_object(seed: int = 0, n: int = 16384) -> Obj:
    """Superquadric with semi-axes U[30,80] mm and exponents U[0.3,2.0];
    area-uniform points by parametric oversampling and area-weighted
    resampling; analytic normals."""
    rng = _rng(seed, _TAG_OBJ)
    a, b, c = rng.uniform(0.030, 0.080, size=3)
    e1, e2 = rng.uniform(0.3, 2.0, size=2)
    eta, om = _sq_area_uniform(rng, a, b, c, e1, e2, n)
    p = _sq_surface(a, b, c, e1, e2, eta, om)
    ce, se, co, so = np.cos(eta), np.sin(eta), np.cos(om), np.sin(om)
    nn = np.stack([_spow(ce, 2 - e1) * _spow(co, 2 - e2) / a,
                   _spow(ce, 2 - e1) * _spow(so, 2 - e2) / b,
                   _spow(se, 2 - e1) / c], axis=1)
    bad = np.linalg.norm(nn, axis=1) < 1e-12
    nn[bad] = p[bad]
    return _finish_object(p, nn, "superquadric",
                          {"axes": (a, b, c), "exponents": (e1, e2)})


# --- tool-like union of ellipsoids and capsules ---------------------------
def _rand_rot(rng) -> np.ndarray:
    q = _shoemake(rng.uniform(size=3))
    return _quat_to_R(q)


def _shoemake(u: np.ndarray) -> np.ndarray:
    """Uniform unit quaternion (w, x, y, z) from three U[0,1) numbers (Shoemake 1992)."""
    u1, u2, u3 = u[..., 0], u[..., 1], u[..., 2]
    a, b = np.sqrt(1.0 - u1), np.sqrt(u1)
    x = a * np.sin(2 * math.pi * u2)
    y = a * np.cos(2 * math.pi * u2)
    z = b * np.sin(2 * math.pi * u3)
    w = b * np.cos(2 * math.pi * u3)
    return np.stack([w, x, y, z], axis=-1)


def _quat_to_R(q: np.ndarray) -> np.ndarray:
    w, x, y, z = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    R = np.stack([
        1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
        2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
        2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], axis=-1)
    return R.reshape(q.shape[:-1] + (3, 3))


class _Capsule:
    def __init__(self, a, b, r):
        self.a, self.b, self.r = np.asarray(a, float), np.asarray(b, float), float(r)

    def area(self):
        return 2 * math.pi * self.r * np.linalg.norm(self.b - self.a) + 4 * math.pi * self.r ** 2

    def sdf(self, x):
        ab = self.b - self.a
        t = np.clip(((x - self.a) @ ab) / (ab @ ab), 0.0, 1.0)
        c = self.a + t[:, None] * ab
        return np.linalg.norm(x - c, axis=1) - self.r

    def sample(self, rng, m):
        ab = self.b - self.a
        L = np.linalg.norm(ab)
        axis = ab / L
        tmp = np.array([1.0, 0, 0]) if abs(axis[0]) < 0.9 else np.array([0, 1.0, 0])
        e1 = np.cross(axis, tmp); e1 /= np.linalg.norm(e1)
        e2 = np.cross(axis, e1)
        a_cyl = 2 * math.pi * self.r * L
        a_sph = 4 * math.pi * self.r ** 2
        u = rng.uniform(size=m)
        cyl = u < a_cyl / (a_cyl + a_sph)
        out_p = np.empty((m, 3)); out_n = np.empty((m, 3))
        k = int(cyl.sum())
        t = rng.uniform(0, L, size=k); ph = rng.uniform(0, 2 * math.pi, size=k)
        nn = np.cos(ph)[:, None] * e1 + np.sin(ph)[:, None] * e2
        out_p[cyl] = self.a + t[:, None] * axis + self.r * nn
        out_n[cyl] = nn
        k2 = m - k
        d = rng.normal(size=(k2, 3)); d /= np.linalg.norm(d, axis=1, keepdims=True)
        cen = np.where(((d @ axis) > 0)[:, None], self.b, self.a)
        out_p[~cyl] = cen + self.r * d
        out_n[~cyl] = d
        return out_p, out_n


class _Ellipsoid:
    def __init__(self, c, R, axes):
        self.c, self.R, self.ax = np.asarray(c, float), np.asarray(R, float), np.asarray(axes, float)

    def area(self):
        a, b, c = self.ax
        p = 1.6075  # Knud Thomsen's approximation
        return 4 * math.pi * (((a * b) ** p + (a * c) ** p + (b * c) ** p) / 3) ** (1 / p)

    def inside(self, x):
        y = (x - self.c) @ self.R
        return ((y / self.ax) ** 2).sum(axis=1) < 1.0

    def sdf(self, x):
        # used only to reject samples inside other primitives (sign matters)
        y = (x - self.c) @ self.R
        k0 = np.linalg.norm(y / self.ax, axis=1)
        k1 = np.linalg.norm(y / self.ax ** 2, axis=1)
        return np.where(k1 > 0, k0 * (k0 - 1.0) / np.maximum(k1, 1e-30), -self.ax.min())

    def sample(self, rng, m):
        # uniform on the sphere, mapped, then area-factor rejection
        out_p, out_n = [], []
        need = m
        amax = max(self.ax[0] * self.ax[1], self.ax[0] * self.ax[2], self.ax[1] * self.ax[2])
        while need > 0:
            d = rng.normal(size=(2 * need + 16, 3)); d /= np.linalg.norm(d, axis=1, keepdims=True)
            g = d / self.ax  # gradient direction in local frame (unnormalised)
            fac = np.linalg.norm(g, axis=1) * self.ax.prod()  # local area scale
            keep = rng.uniform(size=d.shape[0]) * amax < fac
            d, g = d[keep][:need], g[keep][:need]
            out_p.append(self.c + (d * self.ax) @ self.R.T)
            gn = g / np.linalg.norm(g, axis=1, keepdims=True)
            out_n.append(gn @ self.R.T)
            need -= d.shape[0]
        return np.concatenate(out_p), np.concatenate(out_n)


def _tool_primitives(seed: int):
    rng = _rng(seed, _TAG_OBJ)
    L = rng.uniform(0.080, 0.160)
    rh = rng.uniform(0.008, 0.015)
    prims = [_Capsule((-L / 2, 0, 0), (L / 2, 0, 0), rh)]
    head_axes = rng.uniform(0.015, 0.030, size=3)
    prims.append(_Ellipsoid((L / 2 + 0.5 * head_axes[0], 0, 0), _rand_rot(rng), head_axes))
    n_extra = int(rng.integers(0, 5))  # 2..6 primitives in total
    for i in range(n_extra):
        if i % 2 == 0:
            c = np.array([rng.uniform(-L / 2, L / 2 + head_axes[0]),
                          rng.uniform(-0.01, 0.01), rng.uniform(-0.01, 0.01)])
            prims.append(_Ellipsoid(c, _rand_rot(rng), rng.uniform(0.008, 0.025, size=3)))
        else:
            a = np.array([rng.uniform(-L / 2, L / 2), 0.0, 0.0])
            d = rng.normal(size=3); d /= np.linalg.norm(d)
            prims.append(_Capsule(a, a + rng.uniform(0.02, 0.06) * d, rng.uniform(0.005, 0.012)))
    return prims


def _union_surface(prims, rng, m):
    areas = np.array([p.area() for p in prims])
    counts = np.maximum(1, np.round(m * areas / areas.sum()).astype(int))
    P, Nn = [], []
    for i, pr in enumerate(prims):
        p, n = pr.sample(rng, int(counts[i]))
        ok = np.ones(p.shape[0], bool)
        for j, other in enumerate(prims):
            if j != i:
                ok &= other.sdf(p) > 0.0
        P.append(p[ok]); Nn.append(n[ok])
    return np.concatenate(P), np.concatenate(Nn)


def tool_object(seed: int = 0, n: int = 65536) -> Obj:
    """Tool-like union of 2-6 ellipsoids and capsules: a handle capsule
    80-160 mm long and an ellipsoidal head 30-60 mm across, plus extras.
    Points are area-uniform on the union surface; normals from the active
    primitive."""
    prims = _tool_primitives(seed)
    rng = _rng(seed, _TAG_OBJ + 1000)
    p, nn = _union_surface(prims, rng, 3 * n)
    pick = rng.choice(p.shape[0], size=n, replace=False)
    p, nn = p[pick], nn[pick]
    shift = p.mean(axis=0)
    obj = _finish_object(p - shift, nn, "tool", {"shift": shift, "seed": seed})
    return obj


# --------------------------------------------------------------------------
# signed-distance grids of the objects (object frame)
# --------------------------------------------------------------------------
@dataclass
class SDF:
    origin: np.ndarray   # float32 [3], position of node (0,0,0)
    h: float             # node spacing
    dims: int            # G nodes per axis
    values: np.ndarray   # float32 [G,G,G] indexed [iz][iy][ix]


def _sdf_grid_frame(pts: np.ndarray, dims: int, h_min: float, margin: float):
    lo, hi = pts.min(axis=0), pts.max(axis=0)
    ext = float((hi - lo).max()) + 2.0 * margin
    h = max(h_min, ext / (dims - 1))
    centre = 0.5 * (lo + hi)
    origin = centre - 0.5 * h * (dims - 1)
    return origin, h


def _grid_nodes(origin, h, dims):
    ax = np.arange(dims, dtype=np.float64) * h
    z, y, x = np.meshgrid(ax, ax, ax, indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1) + origin


def sdf_sphere(radius: float, dims: int = 64, h_min: float = 0.002, margin: float = 0.011) -> SDF:
    pts = np.array([[-radius] * 3, [radius] * 3])
    origin, h = _sdf_grid_frame(pts, dims, h_min, margin)
    x = _grid_nodes(origin, h, dims)
    v = np.linalg.norm(x, axis=1) - radius
    return SDF(origin.astype(np.float32), float(np.float32(h)), dims,
               v.reshape(dims, dims, dims).astype(np.float32))


# |SDF| is truncated at SDF_CAP (m).  Penetration decisions are unaffected as
# long as (capsule radius - margin) + cell diagonal < SDF_CAP: with r <= 9 mm,
# a 2 mm margin and cells of at most 3.5 mm that is 7 + 6.1 = 13.1 mm.
SDF_CAP = 0.015


def _sdf_from_dense(surface: np.ndarray, inside_fn, pts_bbox, dims, h_min, margin, workers=8) -> SDF:
    """Truncated signed distance on a dims^3 node grid: distance to the nearest
    dense surface sample (capped at SDF_CAP), negative inside."""
    from scipy.spatial import cKDTree
    origin, h = _sdf_grid_frame(pts_bbox, dims, h_min, margin)
    x = _grid_nodes(origin, h, dims)
    dist, _ = cKDTree(surface).query(x, workers=workers, distance_upper_bound=SDF_CAP)
    dist = np.minimum(dist, SDF_CAP)
    sgn = np.where(inside_fn(x), -1.0, 1.0)
    return SDF(origin.astype(np.float32), float(np.float32(h)), dims,
               (sgn * dist).reshape(dims, dims, dims).astype(np.float32))


def sdf_tool(seed: int, obj: Obj, dims: int = 64, h_min: float = 0.002, margin: float = 0.011) -> SDF:
    prims = _tool_primitives(seed)
    shift = obj.params["shift"]
    rng = _rng(seed, _TAG_SDF)
    dense, _ = _union_surface(prims, rng, 600_000)
    dense = dense - shift

    def inside(x):
        xs = x + shift
        ins = np.zeros(x.shape[0], bool)
        for pr in prims:
            ins |= pr.sdf(xs) < 0.0
        return ins
    return _sdf_from_dense(dense, inside, obj.pts.astype(np.float64), dims, h_min, margin)


def sdf_superquadric(obj: Obj, dims: int = 64, h_min: float = 0.002, margin: float = 0.011,
                     n_dense: int = 65536, workers: int = 8) -> SDF:
    """Truncated SDF of a superquadric from n_dense area-weighted surface
    samples (mean spacing about 1 mm at the largest axes; at the 7 mm
    decision distance the nearest-sample distance is within 0.05 mm)."""
    a, b, c = obj.params["axes"]
    e1, e2 = obj.params["exponents"]
    rng = _rng(0, _TAG_SDF)
    eta, om = _sq_area_uniform(rng, a, b, c, e1, e2, n_dense, replace=True)
    dense = _sq_surface(a, b, c, e1, e2, eta, om)

    def inside(x):
        f = (np.abs(x[:, 0] / a) ** (2 / e2) + np.abs(x[:, 1] / b) ** (2 / e2)) ** (e2 / e1) \
            + np.abs(x[:, 2] / c) ** (2 / e1)
        return f < 1.0
    return _sdf_from_dense(dense, inside, obj.pts.astype(np.float64), dims, h_min, margin, workers)


# --------------------------------------------------------------------------
# palm poses
# --------------------------------------------------------------------------
def palm_poses(n: int, seed: int = 0, d_lo: float = 0.08, d_hi: float = 0.12) -> np.ndarray:
    """Object poses in the hand frame, float32 [n,12] = 3x4 [R | t].

    R is uniform on SO(3) (Shoemake); the object origin sits at distance
    d ~ U[d_lo, d_hi] along a direction uniform on the palm's outward (+z)
    hemisphere."""
    rng = _rng(seed, _TAG_POSE)
    R = _quat_to_R(_shoemake(rng.uniform(size=(n, 3))))
    d = rng.uniform(d_lo, d_hi, size=n)
    cz = rng.uniform(0.0, 1.0, size=n)
    ph = rng.uniform(0.0, 2.0 * math.pi, size=n)
    sz = np.sqrt(1.0 - cz * cz)
    u = np.stack([sz * np.cos(ph), sz * np.sin(ph), cz], axis=1)
    t = d[:, None] * u
    M = np.zeros((n, 3, 4))
    M[:, :, :3] = R
    M[:, :, 3] = t
    return M.reshape(n, 12).astype(np.float32)


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------
@dataclass
class SearchParams:
    draws: int          # D draws per pose
    k: int              # contacts per set (one per finger)
    mu: float           # friction coefficient
    m_edges: int        # linearised cone edges
    eps: float          # stability threshold on t*
    seed: int           # Philox key for draws
    request_id: int = 0
    pose_offset: int = 0
    moment_scale: float = 1.0
    opt_outer: int = 0       # rounds of contact-point optimisation (0 = score the draws as drawn)
    opt_inner: int = 8       # candidates per contact and round
    opt_sigma: float = 0.004  # m, std of the tangent-plane mutations


@dataclass
class IKParams:
    iters: int = 10
    phase1: int = 5
    lam: float = 1e-2
    beta: float = 0.01
    tol_pos: float = 0.002
    tol_ang: float = 0.35
    margin: float = 0.002
    self_collision: int = 0   # also reject grasps whose links of different fingers penetrate


@dataclass
class Workload:
    name: str
    hand: Hand
    field: FieldParams
    obj: Obj
    poses: np.ndarray
    search: SearchParams
    ik: Optional[IKParams]
    sdf: Optional[SDF]


def workload(name: str, *, seed: int = 0, n_points: Optional[int] = None,
             n_poses: Optional[int] = None, samples: Optional[int] = None,
             draws: Optional[int] = None, with_sdf: Optional[bool] = None) -> Workload:
    """Build one of the named workloads ``c1``, ``c2``, ``c3``.

    Overrides keep the workload's structure while shrinking a dimension."""
    if name == "c1":
        hand = hand_c1()
        G, h, B, S = 32, 0.004, 32, 8192
        obj = sphere_object(0.04, n_points or 2048)
        P, D, k = 256, 16, 3
        sdf = sdf_sphere(0.04) if with_sdf else None
        ik = IKParams() if with_sdf else None
    elif name == "c2":
        hand = hand_c2(seed)
        G, h, B, S = 64, 0.003, 64, 262144
        obj = superquadric_object(seed, n_points or 16384)
        P, D, k = 16384, 32, 4
        sdf = sdf_superquadric(obj) if with_sdf else None
        ik = IKParams() if with_sdf else None
    elif name == "c3":
        hand = hand_c3(seed)
        G, h, B, S = 64, 0.003, 64, 262144
        obj = tool_object(seed, n_points or 65536)
        P, D, k = 65536, 64, 5
        with_sdf = True if with_sdf is None else with_sdf
        sdf = sdf_tool(seed, obj) if with_sdf else None
        ik = IKParams() if with_sdf else None
    else:
        raise ValueError(f"unknown workload {name!r}")
    P = n_poses or P
    S = samples or S
    D = draws or D
    fp = FieldParams(samples=S, seed=seed, grid=G, h=h, bins=B, grid_frame=grid_frames(hand, G, h))
    sp = SearchParams(draws=D, k=k, mu=0.5, m_edges=8, eps=1e-3, seed=seed, moment_scale=obj.rho)
    return Workload(name=name, hand=hand, field=fp, obj=obj, poses=palm_poses(P, seed),
                    search=sp, ik=ik, sdf=sdf)
