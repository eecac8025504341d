"""FP64 CPU oracle of the Contact-Field pipeline -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path (the HIP library in
``paper_2511_07418_amd``) never does, and the two share no code: the oracle
is ``oracle.c`` (plain C11, double precision, OpenMP over independent work)
plus thin ctypes marshalling here.

Each function cites the passage of the paper it follows (arXiv 2511.07418):

* ``philox``           Philox4x32-10 counter RNG (Salmon et al., SC'11)
* ``joint_sample``     random joint configurations of Sec. 4.3
* ``fk``               forward kinematics F of Sec. 3.1
* ``build_field``      Sec. 4.3 Alg. 1 (grid cover + normals per box) with
                       per-link (patch) tables of Sec. 4.4 and quantised normals
* ``query``            object contact query of Sec. 4.3 and the merged
                       per-dependency-group domains of Sec. 5.3
* ``query_cone``       the theta_hit test of Sec. 4.3 over the field's bin
                       centres (cone query)
* ``draw``             Sec. 5.3 random selection + reverse lookup of Sec. 5.5
* ``verdicts``/``set_tstar``  Eq. 1-2 with a linearised friction cone (LP)
* ``place_exhaustive`` Sec. 5.1 exhaustive placement (object point onto a
                       random contact vector of the field)
* ``optimize``         Sec. 5.4 Alg. 2 (blockwise zeroth-order contact-point
                       optimisation), with ``project_domain`` and ``opt_noise``
* ``relink``           the reverse lookup of Sec. 5.5 for optimised sets
* ``compact``          accepted sets in pose-major, draw-minor order
* ``realize``          Sec. 5.5 Eq. 7-8 (DLS IK with Phase-II projection) and
                       the penetration criterion of Sec. 3.2, optionally with the
                       hand self-collision filter of Sec. 5.6 (``self_penetration``)

Readings where the paper is silent are listed in the design doc.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

BAND = 1e-6


def build(force: bool = True) -> str:
    """Compile ``liboracle.so`` with gcc (plain IEEE double, no contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
               "-Wall", "-shared", "-fPIC", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Hand(C.Structure):
    _fields_ = [("n_fingers", C.c_int32), ("n_joints", C.c_int32),
                ("joint_finger", C.c_void_p), ("joint_parent", C.c_void_p),
                ("joint_origin", C.c_void_p), ("joint_axis", C.c_void_p),
                ("capsule", C.c_void_p), ("limits", C.c_void_p),
                ("n_surf", C.c_int32), ("surf", C.c_void_p)]


class _FieldParams(C.Structure):
    _fields_ = [("samples", C.c_int64), ("seed", C.c_uint64), ("grid", C.c_int32),
                ("h", C.c_double), ("bins", C.c_int32), ("grid_frame", C.c_void_p)]


class _IK(C.Structure):
    _fields_ = [("iters", C.c_int32), ("phase1", C.c_int32), ("lam", C.c_double), ("beta", C.c_double),
                ("tol_pos", C.c_double), ("tol_ang", C.c_double), ("margin", C.c_double),
                ("self_collision", C.c_int32)]


class _SDF(C.Structure):
    _fields_ = [("origin", C.c_double * 3), ("h", C.c_double), ("dims", C.c_int32),
                ("values", C.c_void_p)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = C.CDLL(_LIB)
        vp, i32, i64, u64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_double
        L.orc_philox4x32_10.argtypes = [vp, vp, vp]
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_get_threads.restype = C.c_int
        L.orc_joint_sample.argtypes = [vp, u64, C.c_int, i64, vp]
        L.orc_fk.argtypes = [vp, vp, vp]
        L.orc_fk_finger.argtypes = [vp, C.c_int, vp, vp]
        L.orc_bin_centers.argtypes = [C.c_int, vp]
        L.orc_bin.argtypes = [C.c_int, vp, vp, vp]
        L.orc_bin.restype = C.c_int
        L.orc_build_field.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, i64]
        L.orc_build_field.restype = C.c_int
        L.orc_query.argtypes = [vp, vp, vp, vp, vp, i32, vp, i32, vp, vp, vp, vp]
        L.orc_query.restype = C.c_int
        L.orc_query_cone.argtypes = [vp, vp, vp, vp, vp, i32, vp, i32, dbl, vp, vp, vp]
        L.orc_query_cone.restype = C.c_int
        L.orc_draw.argtypes = [vp, vp, vp, vp, vp, i32, vp, i32, vp, vp, i32, i32, u64, C.c_uint32, i64, vp,
                               vp, vp, vp]
        L.orc_draw.restype = C.c_int
        L.orc_tangent_basis.argtypes = [vp, vp, vp]
        L.orc_wrench_matrix.argtypes = [C.c_int, vp, vp, dbl, C.c_int, dbl, vp]
        L.orc_lp_solve.argtypes = [C.c_int, vp, C.c_int, vp, vp]
        L.orc_lp_solve.restype = dbl
        L.orc_set_tstar.argtypes = [C.c_int, vp, vp, dbl, C.c_int, dbl, C.c_int, vp, vp]
        L.orc_set_tstar.restype = dbl
        L.orc_verdicts.argtypes = [vp, vp, i32, i32, vp, dbl, i32, dbl, dbl, i32, vp, vp, vp, vp]
        L.orc_verdicts.restype = C.c_int
        L.orc_rot_align.argtypes = [vp, vp, vp, vp]
        L.orc_place_exhaustive.argtypes = [vp, vp, vp, vp, i32, i32, u64, C.c_uint32, i64, vp, vp]
        L.orc_place_exhaustive.restype = C.c_int
        L.orc_opt_noise.argtypes = [u64, C.c_uint32, i64, C.c_int, C.c_uint32, dbl, vp]
        L.orc_project_domain.argtypes = [vp, i32, vp, vp, vp]
        L.orc_project_domain.restype = i64
        L.orc_choose_fingers.argtypes = [C.c_int, vp, C.c_int, u64, C.c_uint32, i64, C.c_int, vp]
        L.orc_choose_fingers.restype = C.c_int
        L.orc_unused_joints.argtypes = [vp, C.c_int, u64, C.c_uint32, i64, C.c_int, vp]
        L.orc_place_palm.argtypes = [vp, vp, i32, vp, i32, vp, vp, i32, i32, dbl, dbl, u64, C.c_uint32, i64, vp,
                                     vp, vp, vp, i32]
        L.orc_place_palm.restype = C.c_int
        L.orc_optimize.argtypes = [vp, vp, i32, vp, vp, vp, i32, i32, i32, i32, vp, dbl, i32, dbl, i32, i32, dbl,
                                   u64, C.c_uint32, i64, i32, vp, vp]
        L.orc_optimize.restype = C.c_int
        L.orc_optimize_outcomes.argtypes = [vp, vp, i32, vp, vp, vp, i32, i32, i64, i32, vp, dbl, i32, dbl, i32, i32,
                                            dbl, u64, C.c_uint32, i64, i32, i32, vp, vp]
        L.orc_optimize_outcomes.restype = C.c_int
        L.orc_relink.argtypes = [vp, vp, vp, vp, vp, vp, i32, i32, i32, vp, vp, u64, C.c_uint32, i64, vp, vp]
        L.orc_relink.restype = C.c_int
        L.orc_extend.argtypes = [vp, vp, vp, vp, vp, i32, vp, i32, vp, vp, i32, i32, vp, vp, vp, i32, u64,
                                 C.c_uint32, i64, vp, vp, vp]
        L.orc_extend.restype = C.c_int
        L.orc_segment_distance.argtypes = [vp, vp, vp, vp]
        L.orc_segment_distance.restype = dbl
        L.orc_self_penetration.argtypes = [vp, vp]
        L.orc_self_penetration.restype = dbl
        L.orc_ik_finger.argtypes = [vp, C.c_int, C.c_int, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.orc_capsule_aligned_point.argtypes = [vp, vp, C.c_double, vp, vp, C.c_double, vp, vp, vp]
        L.orc_point_jacobian.argtypes = [vp, C.c_int, C.c_int, vp, vp, vp]
        L.orc_sdf_eval.argtypes = [vp, vp]
        L.orc_sdf_eval.restype = dbl
        L.orc_axis_samples.argtypes = [vp, C.c_int]
        L.orc_axis_samples.restype = C.c_int
        L.orc_penetration.argtypes = [vp, vp, vp, vp]
        L.orc_penetration.restype = dbl
        L.orc_concave_filter.argtypes = [vp, vp, vp, i32, dbl, i32, dbl, vp, vp, vp]
        L.orc_concave_filter.restype = C.c_int
        L.orc_realize.argtypes = [vp, vp, vp, vp, vp, vp, i32, vp, i32, vp, vp, i32, i32, vp, i32, vp,
                                  u64, C.c_uint32, i64, vp, vp, vp, vp, vp, vp, vp, vp]
        L.orc_realize.restype = C.c_int
        _lib = L
    return _lib


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


class _Keep:
    """Holds ctypes structures together with the arrays they point to."""

    def __init__(self, struct, arrays):
        self.struct, self.arrays = struct, arrays

    @property
    def ref(self):
        return C.byref(self.struct)


def _hand(h) -> _Keep:
    arrs = [_c(h.joint_finger, np.int32), _c(h.joint_parent, np.int32),
            _c(h.joint_origin, np.float32), _c(h.joint_axis, np.float32),
            _c(h.capsule, np.float32), _c(h.limits, np.float32), _c(h.surf, np.float32)]
    s = _Hand(h.n_fingers, h.n_joints, _p(arrs[0]), _p(arrs[1]), _p(arrs[2]), _p(arrs[3]),
              _p(arrs[4]), _p(arrs[5]), int(h.surf.shape[1]), _p(arrs[6]))
    return _Keep(s, arrs)


def _field(fp) -> _Keep:
    gf = _c(fp.grid_frame, np.float32)
    s = _FieldParams(int(fp.samples), int(fp.seed) & 0xFFFFFFFFFFFFFFFF, int(fp.grid),
                     float(np.float32(fp.h)), int(fp.bins), _p(gf))
    return _Keep(s, [gf])


def _sdf(sdf) -> _Keep:
    v = _c(sdf.values, np.float32)
    s = _SDF((C.c_double * 3)(*[float(x) for x in np.asarray(sdf.origin, np.float32)]),
             float(np.float32(sdf.h)), int(sdf.dims), _p(v))
    return _Keep(s, [v])


def _ik(ik) -> _IK:
    f32 = lambda x: float(np.float32(x))  # the parameters arrive as float32, promoted exactly
    return _IK(int(ik.iters), int(ik.phase1), f32(ik.lam), f32(ik.beta), f32(ik.tol_pos),
               f32(ik.tol_ang), f32(ik.margin), int(getattr(ik, "self_collision", 0)))


# ---------------------------------------------------------------------------
def set_threads(n: int) -> None:
    """Threads of the oracle's parallel loops from now on."""
    lib().orc_set_threads(int(n))


def get_threads() -> int:
    return int(lib().orc_get_threads())


def philox(ctr, key) -> np.ndarray:
    """Philox4x32-10 block for counter ``ctr`` (4 x uint32) and ``key`` (2 x uint32)."""
    c, k = _c(ctr, np.uint32), _c(key, np.uint32)
    out = np.zeros(4, np.uint32)
    lib().orc_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def joint_sample(hand, seed: int, f: int, s: int) -> np.ndarray:
    """Joint values of finger ``f`` for joint sample ``s`` (Sec. 4.3)."""
    H = _hand(hand)
    q = np.zeros(hand.dof[f], np.float64)
    lib().orc_joint_sample(H.ref, int(seed) & 0xFFFFFFFFFFFFFFFF, f, int(s), _p(q))
    return q


def fk(hand, q) -> np.ndarray:
    """Link frames [J,12] (3x4 [R|t], hand frame) for joint vector ``q`` [J]."""
    H = _hand(hand)
    qq = _c(q, np.float64)
    T = np.zeros((hand.n_joints, 12), np.float64)
    lib().orc_fk(H.ref, _p(qq), _p(T))
    return T


def bin_centers(B: int) -> np.ndarray:
    c = np.zeros((B, 3), np.float64)
    lib().orc_bin_centers(B, _p(c))
    return c


def bin_of(B: int, d) -> tuple[int, int, float]:
    """(best bin, second bin, (theta2 - theta1)/2) of direction ``d``."""
    dd = _c(d, np.float64)
    b2 = C.c_int(0)
    gap = C.c_double(0)
    b = lib().orc_bin(B, _p(dd), C.byref(b2), C.byref(gap))
    return b, b2.value, gap.value


def build_field(hand, fp, witness: bool = False, flags: bool = True, sample_ids=None) -> dict:
    """Per-link voxel x normal-bin bit tables (Alg. 1 as a dense grid cover).

    Returns ``bits``/``sure``/``maybe`` uint32 [L, G^3, B/32] and, with
    ``witness``, int32 [L, G^3, B] ``wit``/``wit_lo``/``wit_hi`` (-1 = none),
    plus ``stats`` = (vectors, in-window, dropped, flagged).  ``sample_ids``
    restricts the cover to those joint samples of every finger (default: all
    ``fp.samples``)."""
    G, B, L = fp.grid, fp.bins, hand.n_joints
    shp = (L, G ** 3, B // 32)
    bits = np.zeros(shp, np.uint32)
    sure = np.zeros(shp, np.uint32) if flags else None
    maybe = np.zeros(shp, np.uint32) if flags else None
    wshp = (L, G ** 3, B)
    wit = np.zeros(wshp, np.int32) if witness else None
    wlo = np.zeros(wshp, np.int32) if (witness and flags) else None
    whi = np.zeros(wshp, np.int32) if (witness and flags) else None
    stats = np.zeros(4, np.int64)
    H, Fp = _hand(hand), _field(fp)
    ids = None if sample_ids is None else _c(sample_ids, np.int64)
    if ids is not None and ((ids < 0) | (ids >= fp.samples)).any():
        raise ValueError("sample id outside 0..samples-1")
    rc = lib().orc_build_field(H.ref, Fp.ref, _p(bits), _p(sure), _p(maybe), _p(wit), _p(wlo),
                               _p(whi), _p(stats), _p(ids), 0 if ids is None else len(ids))
    if rc != 0:
        raise ValueError(f"orc_build_field failed ({rc})")
    return {"bits": bits, "sure": sure, "maybe": maybe, "wit": wit, "wit_lo": wlo,
            "wit_hi": whi, "stats": stats}


def query(hand, fp, bits, pts, nrm, poses, flags: bool = True) -> dict:
    """Contact domains: ``dom_bits`` uint32 [P,F,ceil(N/32)], ``dom_count``
    uint32 [P,F], ``dom_flag`` (same shape as bits) and the number of in-window
    (pose, point, link) lookups."""
    pts, nrm, poses = _c(pts, np.float32), _c(nrm, np.float32), _c(poses, np.float32)
    P, N, F = poses.shape[0], pts.shape[0], hand.n_fingers
    NW = (N + 31) // 32
    db = np.zeros((P, F, NW), np.uint32)
    dc = np.zeros((P, F), np.uint32)
    df = np.zeros((P, F, NW), np.uint32) if flags else None
    lk = C.c_int64(0)
    H, Fp = _hand(hand), _field(fp)
    bb = _c(bits, np.uint32)
    rc = lib().orc_query(H.ref, Fp.ref, _p(bb), _p(pts), _p(nrm), N, _p(poses), P, _p(db), _p(dc),
                         _p(df), C.byref(lk))
    if rc != 0:
        raise ValueError(f"orc_query failed ({rc})")
    return {"dom_bits": db, "dom_count": dc, "dom_flag": df, "lookups": lk.value}


def query_cone(hand, fp, bits, pts, nrm, poses, cos_hit: float, flags: bool = True) -> dict:
    """Cone query (Sec. 4.3 theta_hit test over the field's bin centres)."""
    pts, nrm, poses = _c(pts, np.float32), _c(nrm, np.float32), _c(poses, np.float32)
    N, P, F = pts.shape[0], poses.shape[0], hand.n_fingers
    NW = (N + 31) // 32
    db = np.zeros((P, F, NW), np.uint32)
    dc = np.zeros((P, F), np.uint32)
    df = np.zeros((P, F, NW), np.uint32) if flags else None
    H, Fp = _hand(hand), _field(fp)
    rc = lib().orc_query_cone(H.ref, Fp.ref, _p(_c(bits, np.uint32)), _p(pts), _p(nrm), N, _p(poses), P,
                              float(cos_hit), _p(db), _p(dc), _p(df))
    if rc != 0:
        raise ValueError(f"orc_query_cone failed ({rc})")
    return {"dom_bits": db, "dom_count": dc, "dom_flag": df}


def draw(hand, fp, bits, pts, nrm, poses, dom_bits, dom_count, sp, palm_pt=None, link_flags: bool = False):
    """Seeded contact-set draws: ``set_pt``, ``set_link`` int32 [P, D, k]
    (none for poses whose palm placement was rejected, ``palm_pt == -2``).
    With ``link_flags`` a third array uint8 [P, D, k] marks links decided
    inside a rounding band (voxel face within 1e-6 m or bin boundary within
    1e-6 rad, with another link on the other side)."""
    pts, nrm, poses = _c(pts, np.float32), _c(nrm, np.float32), _c(poses, np.float32)
    P, N = poses.shape[0], pts.shape[0]
    spt = np.zeros((P, sp.draws, sp.k), np.int32)
    sln = np.zeros((P, sp.draws, sp.k), np.int32)
    lfl = np.zeros((P, sp.draws, sp.k), np.uint8) if link_flags else None
    H, Fp = _hand(hand), _field(fp)
    rc = lib().orc_draw(H.ref, Fp.ref, _p(_c(bits, np.uint32)), _p(pts), _p(nrm), N, _p(poses), P,
                        _p(_c(dom_bits, np.uint32)), _p(_c(dom_count, np.uint32)), sp.draws, sp.k,
                        int(sp.seed) & 0xFFFFFFFFFFFFFFFF, int(sp.request_id), int(sp.pose_offset),
                        _p(None if palm_pt is None else _c(palm_pt, np.int32)), _p(spt), _p(sln), _p(lfl))
    if rc != 0:
        raise ValueError(f"orc_draw failed ({rc})")
    return (spt, sln, lfl) if link_flags else (spt, sln)


def tangent_basis(n) -> tuple[np.ndarray, np.ndarray]:
    nn = _c(n, np.float64)
    x, y = np.zeros(3), np.zeros(3)
    lib().orc_tangent_basis(_p(nn), _p(x), _p(y))
    return x, y


def wrench_matrix(p, n, mu: float, m: int, rho: float) -> np.ndarray:
    """Wrench columns [k*m, 6] of the linearised cones."""
    p, n = _c(p, np.float64), _c(n, np.float64)
    k = p.shape[0]
    W = np.zeros((k * m, 6), np.float64)
    lib().orc_wrench_matrix(k, _p(p), _p(n), float(mu), int(m), float(rho), _p(W))
    return W


def lp_solve(W, max_pivots: int = 1000) -> tuple[float, int, int]:
    """t* = min ||W^T g||_1 over the simplex; returns (t*, status, pivots)."""
    W = _c(W, np.float64)
    st, pv = C.c_int(0), C.c_int(0)
    t = lib().orc_lp_solve(W.shape[0], _p(W), int(max_pivots), C.byref(st), C.byref(pv))
    return t, st.value, pv.value


def set_tstar(p, n, mu: float, m: int, rho: float, max_pivots: int = 1000) -> tuple[float, int]:
    p, n = _c(p, np.float64), _c(n, np.float64)
    st, pv = C.c_int(0), C.c_int(0)
    t = lib().orc_set_tstar(p.shape[0], _p(p), _p(n), float(mu), int(m), float(rho),
                            int(max_pivots), C.byref(st), C.byref(pv))
    return t, st.value


def verdicts(pts, nrm, set_pt, sp, max_pivots: int = 1000) -> dict:
    """Force-closure verdicts of drawn sets (object frame)."""
    pts, nrm = _c(pts, np.float32), _c(nrm, np.float32)
    sets = _c(set_pt, np.int32).reshape(-1, sp.k)
    n = sets.shape[0]
    v = np.zeros(n, np.uint8)
    t = np.zeros(n, np.float64)
    vf = np.zeros(n, np.uint8)
    st = np.zeros(n, np.int32)
    rc = lib().orc_verdicts(_p(pts), _p(nrm), n, sp.k, _p(sets), float(np.float32(sp.mu)),
                            sp.m_edges, float(np.float32(sp.moment_scale)),
                            float(np.float32(sp.eps)), int(max_pivots), _p(v), _p(t), _p(vf),
                            _p(st))
    if rc != 0:
        raise ValueError(f"orc_verdicts failed ({rc})")
    return {"verdict": v, "tstar": t, "vflag": vf, "status": st}


def rot_align(a, b) -> np.ndarray:
    """Rotation [3, 3] taking the direction of a onto the direction of b."""
    R = np.zeros(9)
    lib().orc_rot_align(_p(_c(a, np.float64)), _p(_c(b, np.float64)), _p(R), None)
    return R.reshape(3, 3)


def place_exhaustive(hand, fp, pts, nrm, n_poses: int, seed: int, request_id: int = 0,
                     pose_offset: int = 0) -> dict:
    """Sec. 5.1 exhaustive placement: poses [P, 12] (float64) and near-branch flags."""
    pts, nrm = _c(pts, np.float32), _c(nrm, np.float32)
    out = np.zeros((n_poses, 12), np.float64)
    fl = np.zeros(n_poses, np.uint8)
    H, Fp = _hand(hand), _field(fp)
    rc = lib().orc_place_exhaustive(H.ref, Fp.ref, _p(pts), _p(nrm), pts.shape[0], int(n_poses),
                                    int(seed) & 0xFFFFFFFFFFFFFFFF, int(request_id), int(pose_offset),
                                    _p(out), _p(fl))
    if rc != 0:
        raise ValueError(f"orc_place_exhaustive failed ({rc})")
    return {"poses": out, "pflag": fl}


def opt_noise(seed: int, request_id: int, g: int, d: int, step: int, sigma: float) -> np.ndarray:
    """Tangent-plane offsets (dx, dy) of one candidate of Sec. 5.4 Alg. 2."""
    out = np.zeros(2, np.float64)
    lib().orc_opt_noise(int(seed) & 0xFFFFFFFFFFFFFFFF, int(request_id), int(g), int(d), int(step),
                        float(sigma), _p(out))
    return out


def project_domain(pts, dom_words, y) -> tuple[int, bool]:
    """Nearest point of a contact domain (bitset over points) to y; (index, near-tie flag)."""
    pts = _c(pts, np.float32)
    yy = _c(y, np.float64)
    fl = C.c_int(0)
    i = lib().orc_project_domain(_p(pts), pts.shape[0], _p(_c(dom_words, np.uint32)), _p(yy), C.byref(fl))
    return int(i), bool(fl.value)


def _dom_count(dom_count, dom_bits, P: int, F: int) -> np.ndarray:
    if dom_count is not None:
        return _c(dom_count, np.uint32).reshape(P, F)
    # the domains' sizes, counted from their bitsets
    b = np.ascontiguousarray(dom_bits, np.uint32).reshape(P, F, -1)
    return np.unpackbits(b.view(np.uint8), axis=-1).sum(-1).astype(np.uint32)


def choose_fingers(dom_count, k: int, sp, draws: Optional[int] = None) -> np.ndarray:
    """Contact fingers [P, D, k] of every set (-1 where fewer than k domains are non-empty)."""
    cnt = _c(dom_count, np.uint32)
    P, F = cnt.shape
    D = sp.draws if draws is None else int(draws)
    out = np.full((P, D, k), -1, np.int32)
    row = np.zeros(k, np.int32)
    for g in range(P):
        for d in range(D):
            if lib().orc_choose_fingers(F, _p(cnt[g]), int(k), int(sp.seed) & 0xFFFFFFFFFFFFFFFF,
                                        int(sp.request_id), int(sp.pose_offset) + g, d, _p(row)):
                out[g, d] = row
    return out


def unused_joints(hand, f: int, sp, g: int, d: int) -> np.ndarray:
    """Random joint values [dof] of finger f when it carries no contact of set (g, d)."""
    q = np.zeros(hand.n_joints)
    H = _hand(hand)
    lib().orc_unused_joints(H.ref, int(f), int(sp.seed) & 0xFFFFFFFFFFFFFFFF, int(sp.request_id),
                            int(sp.pose_offset) + int(g), int(d), _p(q))
    j = np.flatnonzero(np.asarray(hand.joint_finger) == f)
    return q[j]


def optimize(pts, nrm, dom_bits, set_pt, sp, F: int, max_pivots: int = 1000, dom_count=None,
             palm_pt=None) -> dict:
    """Sec. 5.4 Alg. 2 on drawn sets: optimised set_pt [P, D, k], t* of the final
    sets (NaN for invalid draws) and the band flag of each set.  ``dom_count``
    (default: the domains' popcounts) decides the sets' fingers."""
    pts, nrm = _c(pts, np.float32), _c(nrm, np.float32)
    spt = _c(set_pt, np.int32).copy()
    P, D, k = spt.shape
    t = np.zeros(P * D, np.float64)
    fl = np.zeros(P * D, np.uint8)
    cnt = _dom_count(dom_count, dom_bits, P, int(F))
    palm = None if palm_pt is None else _c(palm_pt, np.int32)
    rc = lib().orc_optimize(_p(pts), _p(nrm), pts.shape[0], _p(_c(dom_bits, np.uint32)), _p(cnt), _p(palm), P,
                            int(F), D, k,
                            _p(spt), float(np.float32(sp.mu)), sp.m_edges, float(np.float32(sp.moment_scale)),
                            int(sp.opt_outer), int(sp.opt_inner), float(np.float32(sp.opt_sigma)),
                            int(sp.seed) & 0xFFFFFFFFFFFFFFFF, int(sp.request_id), int(sp.pose_offset),
                            int(max_pivots), _p(t), _p(fl))
    if rc != 0:
        raise ValueError(f"orc_optimize failed ({rc})")
    eps = float(np.float32(sp.eps))
    return {"set_pt": spt, "tstar": t, "oflag": fl, "verdict": (t <= eps).astype(np.uint8),
            "vflag": (np.abs(t - eps) <= BAND).astype(np.uint8)}


def optimize_outcomes(pts, nrm, dom_bits, set_pt, sp, F: int, sets, max_pivots: int = 1000, dom_count=None,
                      palm_pt=None, max_out: int = 64) -> list:
    """Every outcome of Alg. 2 (Sec. 5.4) the rounding bands admit, for each flat
    set id in ``sets`` of the drawn ``set_pt`` [P, D, k]: a list of (points
    [n, k], J [n]) pairs, where n = 0 for a set that is not valid and None
    when more than ``max_out`` outcomes exist.  ``optimize``'s result is always
    one of them, and the only one for a set it does not flag."""
    pts, nrm = _c(pts, np.float32), _c(nrm, np.float32)
    spt = _c(set_pt, np.int32)
    P, D, k = spt.shape
    cnt = _dom_count(dom_count, dom_bits, P, int(F))
    bits = _c(dom_bits, np.uint32)
    palm = None if palm_pt is None else _c(palm_pt, np.int32)
    out = []
    for s in np.asarray(sets, np.int64):
        g, d = int(s) // D, int(s) % D
        opt = np.zeros((max_out, k), np.int32)
        ot = np.zeros(max_out, np.float64)
        start = np.ascontiguousarray(spt[g, d])
        n = lib().orc_optimize_outcomes(_p(pts), _p(nrm), pts.shape[0], _p(bits), _p(cnt), _p(palm), int(F), k, g, d,
                                        _p(start), float(np.float32(sp.mu)), sp.m_edges,
                                        float(np.float32(sp.moment_scale)), int(sp.opt_outer), int(sp.opt_inner),
                                        float(np.float32(sp.opt_sigma)), int(sp.seed) & 0xFFFFFFFFFFFFFFFF,
                                        int(sp.request_id), int(sp.pose_offset), int(max_pivots), int(max_out),
                                        _p(opt), _p(ot))
        if n < -1:
            raise ValueError("orc_optimize_outcomes: bad parameters")
        out.append(None if n < 0 else (opt[:n].copy(), ot[:n].copy()))
    return out


def verdicts_palm(pts, nrm, set_pt, palm_pt, sp, max_pivots: int = 1000) -> dict:
    """Verdicts of drawn sets with each pose's palm contact (Sec. 5.1 static
    link) as one more contact: sets of poses with palm_pt >= 0 are scored with
    k + 1 contacts, the others with their k."""
    spt = _c(set_pt, np.int32)
    P, D, k = spt.shape
    palm = _c(palm_pt, np.int32)
    out = {"verdict": np.zeros(P * D, np.uint8), "tstar": np.full(P * D, np.nan),
           "vflag": np.zeros(P * D, np.uint8), "status": np.zeros(P * D, np.int32)}
    with_palm = palm >= 0
    for mask, kk in ((with_palm, k + 1), (~with_palm, k)):
        g = np.flatnonzero(mask)
        if len(g) == 0:
            continue
        sets = spt[g]
        if kk > k:
            sets = np.concatenate([sets, np.broadcast_to(palm[g][:, None, None], (len(g), D, 1))], axis=2)
            # an undrawn set stays undrawn
            sets = np.where((spt[g] < 0).any(-1, keepdims=True), -1, sets)
        V = verdicts(pts, nrm, np.ascontiguousarray(sets, np.int32), _with_k(sp, kk), max_pivots)
        rows = (g[:, None] * D + np.arange(D)[None, :]).reshape(-1)
        for key in out:
            out[key][rows] = V[key]
    return out


def _with_k(sp, k: int):
    import dataclasses
    return dataclasses.replace(sp, k=int(k))


def place_palm(palm, sdf, pts, nrm, poses, prob: float, margin: float, seed: int, request_id: int = 0,
               pose_offset: int = 0, flip: bool = False) -> dict:
    """Sec. 5.1 static-link placement over ``poses`` [P, 12] (float64 out): the
    palm poses, palm_pt (i / -1 / -2), the selected point sel_pt (i, or -1)
    and the band flags (bit 1: rotation branch, bit 2: penetration at the
    margin).  ``flip`` takes the other rotation branch on bit-1 poses."""
    pts, nrm = _c(pts, np.float32), _c(nrm, np.float32)
    out = np.ascontiguousarray(poses, np.float64).copy()
    P = out.shape[0]
    pp = np.zeros(P, np.int32)
    sel = np.zeros(P, np.int32)
    fl = np.zeros(P, np.uint8)
    S = _sdf(sdf)
    surf, caps = _c(palm.surf, np.float32), _c(palm.caps, np.float32)
    rc = lib().orc_place_palm(S.ref, _p(surf), surf.shape[0], _p(caps), caps.shape[0], _p(pts), _p(nrm),
                              pts.shape[0], P, float(np.float32(prob)), float(np.float32(margin)),
                              int(seed) & 0xFFFFFFFFFFFFFFFF, int(request_id), int(pose_offset), _p(out), _p(pp),
                              _p(fl), _p(sel), int(bool(flip)))
    if rc != 0:
        raise ValueError(f"orc_place_palm failed ({rc})")
    return {"poses": out, "palm_pt": pp, "pflag": fl, "sel_pt": sel}


def relink(hand, fp, bits, pts, nrm, poses, set_pt, sp, dom_count=None, link_flags: bool = False):
    """Links of (optimised) sets, picked with each set's draw words.  ``dom_count``
    decides the sets' fingers; it may be left out when k equals the number of
    fingers (every finger then carries contact i = finger i).  ``link_flags``:
    also return the band flags of ``draw``."""
    pts, nrm, poses = _c(pts, np.float32), _c(nrm, np.float32), _c(poses, np.float32)
    spt = _c(set_pt, np.int32)
    P, D, k = spt.shape
    F = hand.n_fingers
    if dom_count is None:
        if k != F:
            raise ValueError("relink with k < number of fingers needs dom_count")
        dom_count = np.ones((P, F), np.uint32)
    cnt = _c(dom_count, np.uint32).reshape(P, F)
    sln = np.zeros((P, D, k), np.int32)
    lfl = np.zeros((P, D, k), np.uint8) if link_flags else None
    H, Fp = _hand(hand), _field(fp)
    rc = lib().orc_relink(H.ref, Fp.ref, _p(_c(bits, np.uint32)), _p(pts), _p(nrm), _p(poses), P, D, k,
                          _p(cnt), _p(spt), int(sp.seed) & 0xFFFFFFFFFFFFFFFF, int(sp.request_id),
                          int(sp.pose_offset), _p(sln), _p(lfl))
    if rc != 0:
        raise ValueError(f"orc_relink failed ({rc})")
    return (sln, lfl) if link_flags else sln


def extend(hand, fp, bits, pts, nrm, poses, dom_bits, dom_count, set_pt, set_link, take, k_add: int, sp,
           request_id: int = 0) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Second contact round on the unused fingers: ``k_add`` more contacts for
    each round-1 set marked in ``take`` [P, D] (round-1 sets ``set_pt``,
    ``set_link`` [P, D, k1] of the search ``sp``: its seed and pose offset key
    the draws, ``request_id`` is this round's).  Returns the extended sets
    ``set_pt``, ``set_link`` int32 [P, D, k1 + k_add] (all -1 where not
    extended) and the new links' band flags (see ``draw``)."""
    pts, nrm, poses = _c(pts, np.float32), _c(nrm, np.float32), _c(poses, np.float32)
    s1, l1 = _c(set_pt, np.int32), _c(set_link, np.int32)
    P, D, k1 = s1.shape
    k2 = k1 + int(k_add)
    spt = np.zeros((P, D, k2), np.int32)
    sln = np.zeros((P, D, k2), np.int32)
    lfl = np.zeros((P, D, k2), np.uint8)
    H, Fp = _hand(hand), _field(fp)
    rc = lib().orc_extend(H.ref, Fp.ref, _p(_c(bits, np.uint32)), _p(pts), _p(nrm), pts.shape[0], _p(poses), P,
                          _p(_c(dom_bits, np.uint32)), _p(_c(dom_count, np.uint32)), D, k1, _p(s1), _p(l1),
                          _p(_c(np.asarray(take).reshape(P, D), np.uint8)), int(k_add),
                          int(sp.seed) & 0xFFFFFFFFFFFFFFFF, int(request_id), int(sp.pose_offset), _p(spt),
                          _p(sln), _p(lfl))
    if rc != 0:
        raise ValueError(f"orc_extend failed ({rc})")
    return spt, sln, lfl


def compact(verdict) -> np.ndarray:
    """Accepted set ids (g*D + d) in pose-major, draw-minor order."""
    return np.flatnonzero(np.asarray(verdict).reshape(-1)).astype(np.int32)


def ik_finger(hand, f: int, link: int, p, n, q0, ik) -> dict:
    H = _hand(hand)
    q = _c(q0, np.float64).copy()
    pp, nn = _c(p, np.float64), _c(n, np.float64)
    err, ang, gap = C.c_double(0), C.c_double(0), C.c_double(0)
    pt, nt = np.zeros(3), np.zeros(3)
    ikp = _ik(ik)
    lib().orc_ik_finger(H.ref, f, link, _p(pp), _p(nn), C.byref(ikp), _p(q), C.byref(err),
                        C.byref(ang), _p(pt), _p(nt), C.byref(gap))
    return {"q": q, "err": err.value, "ang": ang.value, "pt": pt, "nt": nt, "choice_gap": gap.value}


def capsule_aligned_point(a, b, r: float, p, n, beta: float) -> dict:
    """Point of the capsule (axis a-b, radius r) of least |x - p|^2 + beta^2 |nt - n|^2
    (the hand contact point of the reverse lookup, Sec. 5.5), its outward normal and
    the tie margin of the choice between distant candidates (+inf: none)."""
    a, b, p, n = (_c(v, np.float64) for v in (a, b, p, n))
    pt, nt = np.zeros(3), np.zeros(3)
    gap = C.c_double(0)
    lib().orc_capsule_aligned_point(_p(a), _p(b), float(r), _p(p), _p(n), float(beta), _p(pt), _p(nt),
                                    C.byref(gap))
    return {"pt": pt, "nt": nt, "gap": gap.value}


def point_jacobian(hand, f: int, link: int, q, x) -> np.ndarray:
    """3 x d_f position Jacobian of point ``x`` fixed to ``link`` (Eq. 8)."""
    H = _hand(hand)
    T = fk(hand, q)
    xx = _c(x, np.float64)
    Jm = np.zeros((3, hand.dof[f]), np.float64)
    lib().orc_point_jacobian(H.ref, f, link, _p(T), _p(xx), _p(Jm))
    return Jm


def segment_distance(p1, q1, p2, q2) -> float:
    """Distance between segments [p1, q1] and [p2, q2] (closed form)."""
    a = [_c(v, np.float64) for v in (p1, q1, p2, q2)]
    return float(lib().orc_segment_distance(*[_p(v) for v in a]))


def self_penetration(hand, q) -> float:
    """Deepest penetration between capsules of different fingers at joint vector q (Sec. 5.6)."""
    T = fk(hand, q)
    H = _hand(hand)
    return float(lib().orc_self_penetration(H.ref, _p(_c(T, np.float64))))


def sdf_eval(sdf, y) -> float:
    S = _sdf(sdf)
    yy = _c(y, np.float64)
    return lib().orc_sdf_eval(S.ref, _p(yy))


def axis_samples(hand, l: int) -> int:
    return lib().orc_axis_samples(_hand(hand).ref, l)


def penetration(hand, q, sdf, pose) -> float:
    H, S = _hand(hand), _sdf(sdf)
    T = fk(hand, q)
    pp = _c(pose, np.float32)
    return lib().orc_penetration(H.ref, _p(T), S.ref, _p(pp))


def concave_filter(sdf, pts, nrm, box_edge: float, lattice: int, max_depth: float) -> dict:
    """Sec. 5.2 object preprocessing: per point the penetration depth of a cube of
    edge ``box_edge`` standing on the surface there, keep = depth <= max_depth,
    and the band flag of each decision."""
    pts, nrm = _c(pts, np.float32), _c(nrm, np.float32)
    n = pts.shape[0]
    dep = np.zeros(n)
    keep = np.zeros(n, np.uint8)
    fl = np.zeros(n, np.uint8)
    S = _sdf(sdf)
    rc = lib().orc_concave_filter(S.ref, _p(pts), _p(nrm), n, float(np.float32(box_edge)), int(lattice),
                                  float(np.float32(max_depth)), _p(dep), _p(keep), _p(fl))
    if rc != 0:
        raise ValueError(f"orc_concave_filter failed ({rc})")
    return {"depth": dep, "keep": keep, "flag": fl}


def realize(hand, fp, wit, sdf, pts, nrm, poses, set_pt, set_link, sp, acc_list, ik) -> dict:
    """IK + penetration + acceptance for accepted set ids ``acc_list``."""
    pts, nrm, poses = _c(pts, np.float32), _c(nrm, np.float32), _c(poses, np.float32)
    acc = _c(acc_list, np.int32)
    n, J, k = acc.shape[0], hand.n_joints, sp.k
    q = np.zeros((n, J)); q0 = np.zeros((n, J))
    err = np.zeros((n, k)); ang = np.zeros((n, k)); dep = np.zeros(n)
    val = np.zeros(n, np.uint8); fl = np.zeros(n, np.uint8); mg = np.zeros((n, 3))
    H, Fp, S = _hand(hand), _field(fp), _sdf(sdf)
    ikp = _ik(ik)
    w = None if wit is None else _c(wit, np.int32)
    rc = lib().orc_realize(H.ref, Fp.ref, _p(w), S.ref, _p(pts), _p(nrm), pts.shape[0], _p(poses),
                           poses.shape[0], _p(_c(set_pt, np.int32)), _p(_c(set_link, np.int32)), k, sp.draws,
                           _p(acc), n, C.byref(ikp), int(sp.seed) & 0xFFFFFFFFFFFFFFFF, int(sp.request_id),
                           int(sp.pose_offset), _p(q), _p(q0), _p(err), _p(ang), _p(dep), _p(val), _p(fl),
                           _p(mg))
    if rc != 0:
        raise ValueError(f"orc_realize failed ({rc})")
    return {"q": q, "q0": q0, "contact_err": err, "contact_ang": ang, "depth": dep,
            "valid": val, "rflag": fl, "margin": mg}
