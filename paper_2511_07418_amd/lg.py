"""Thin Python binding of the gfx950 Contact-Field library (``liblg.so``).

Argument marshalling only: every step of the path runs in the library's HIP
kernels.  Functions carry the C ABI's names (``lg_build_field``,
``lg_query_domains``, ``lg_search``, ``lg_realize``, ...).  Device buffers are
``torch`` tensors on the current HIP device; host arrays are NumPy arrays.
If the library has not been built the import of this module raises: there is
no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# LG_LIBRARY names another build of the same library (e.g. a kernel variant under test)
LIB_PATH = os.environ.get("LG_LIBRARY") or os.path.join(_HERE, "liblg.so")

LG_OK, LG_EINVAL, LG_ENOMEM, LG_EDEVICE, LG_EBUDGET, LG_EUNSUPPORTED, LG_EINTERNAL = 0, -1, -2, -3, -4, -5, -6
LG_REQ_QUEUED, LG_REQ_RUNNING, LG_REQ_DONE, LG_REQ_CANCELLED, LG_REQ_FAILED = 0, 1, 2, 3, 4


class LgError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: status {status} ({detail})")
        self.status = status


# ---- C structures (mirror include/lg.h) -------------------------------------
class HandDesc(C.Structure):
    _fields_ = [("n_fingers", C.c_int32), ("n_joints", C.c_int32),
                ("joint_finger", C.c_void_p), ("joint_parent", C.c_void_p),
                ("joint_origin", C.c_void_p), ("joint_axis", C.c_void_p),
                ("capsule", C.c_void_p), ("limits", C.c_void_p),
                ("n_surf", C.c_int32), ("surf", C.c_void_p),
                ("n_palm_surf", C.c_int32), ("palm_surf", C.c_void_p),
                ("n_palm_caps", C.c_int32), ("palm_caps", C.c_void_p)]


class FieldParams(C.Structure):
    _fields_ = [("samples", C.c_int64), ("seed", C.c_uint64), ("grid", C.c_int32),
                ("h", C.c_float), ("bins", C.c_int32), ("grid_frame", C.c_void_p),
                ("keep_witness", C.c_int32)]


class FieldInfo(C.Structure):
    _fields_ = [("n_fingers", C.c_int32), ("n_joints", C.c_int32), ("grid", C.c_int32),
                ("bins", C.c_int32), ("samples", C.c_int64), ("device_bytes", C.c_uint64),
                ("bits_set", C.c_uint64), ("vectors", C.c_int64), ("dropped", C.c_int64),
                ("has_witness", C.c_int32), ("lattice", C.c_int32), ("build_kernel_ms", C.c_double)]


class ExtendParams(C.Structure):
    _fields_ = [("k_add", C.c_int32), ("request_id", C.c_uint32), ("list", C.c_void_p), ("list_n", C.c_void_p),
                ("list_ok", C.c_void_p)]


class SearchParams(C.Structure):
    _fields_ = [("draws", C.c_int32), ("k", C.c_int32), ("m_edges", C.c_int32),
                ("max_pivots", C.c_int32), ("mu", C.c_float), ("eps", C.c_float),
                ("moment_scale", C.c_float), ("seed", C.c_uint64), ("request_id", C.c_uint32),
                ("pose_offset", C.c_int64), ("opt_outer", C.c_int32), ("opt_inner", C.c_int32),
                ("opt_sigma", C.c_float), ("palm_pt", C.c_void_p)]


class IkParams(C.Structure):
    _fields_ = [("iters", C.c_int32), ("phase1", C.c_int32), ("lam", C.c_float),
                ("beta", C.c_float), ("tol_pos", C.c_float), ("tol_ang", C.c_float),
                ("margin", C.c_float), ("self_collision", C.c_int32), ("seed", C.c_uint64),
                ("request_id", C.c_uint32), ("pose_offset", C.c_int64)]


class Sdf(C.Structure):
    _fields_ = [("origin", C.c_float * 3), ("h", C.c_float), ("dims", C.c_int32),
                ("values", C.c_void_p)]


class ServerParams(C.Structure):
    _fields_ = [("budget_bytes", C.c_uint64), ("max_active", C.c_int32), ("chunk_poses", C.c_int32),
                ("batched", C.c_int32), ("batch_slots", C.c_int32)]


class Request(C.Structure):
    _fields_ = [("field", C.c_void_p), ("pts", C.c_void_p), ("nrm", C.c_void_p), ("n_points", C.c_int32),
                ("poses", C.c_void_p), ("n_poses", C.c_int32), ("search", SearchParams),
                ("request_id", C.c_uint32), ("realize", C.c_int32), ("ik", IkParams),
                ("sdf_values", C.c_void_p), ("sdf_origin", C.c_float * 3), ("sdf_h", C.c_float),
                ("sdf_dims", C.c_int32)]


class Result(C.Structure):
    _fields_ = [("state", C.c_int32), ("status", C.c_int32), ("n_acc", C.c_int64), ("n_valid", C.c_int64),
                ("acc_hash", C.c_uint64), ("t_submit", C.c_double), ("t_admit", C.c_double),
                ("t_done", C.c_double), ("bytes", C.c_uint64)]


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("admitted", C.c_int64), ("completed", C.c_int64),
                ("cancelled", C.c_int64), ("rejected", C.c_int64), ("failed", C.c_int64),
                ("budget_bytes", C.c_uint64), ("bytes_in_use", C.c_uint64), ("peak_bytes", C.c_uint64),
                ("queued", C.c_int32), ("active", C.c_int32), ("batches", C.c_int64),
                ("batched_chunks", C.c_int64)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: run paper_2511_07418_amd/build.py "
                          "(or __graft_entry__.build()) first")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
    L.lg_status_str.restype = C.c_char_p
    L.lg_status_str.argtypes = [i32]
    L.lg_last_error.restype = C.c_char_p
    L.lg_version.restype = C.c_char_p
    L.lg_build_field.argtypes = [vp, vp, vp, vp]
    L.lg_field_import.argtypes = [vp, vp, vp, vp, vp]
    L.lg_field_export.argtypes = [vp, vp, vp]
    L.lg_field_info.argtypes = [vp, vp]
    L.lg_field_release.argtypes = [vp]
    L.lg_query_domains.argtypes = [vp, vp, vp, i32, vp, i32, vp, vp, vp]
    L.lg_query_domains_cone.argtypes = [vp, vp, vp, i32, vp, i32, vp, C.c_float, vp, vp, vp]
    L.lg_query_domains_bounded.argtypes = [vp, vp, vp, i32, vp, i32, vp, vp, vp, vp]
    L.lg_chunk_bounds.argtypes = [vp, i32, vp, vp]
    L.lg_morton_order.argtypes = [vp, i32, vp]
    L.lg_search_workspace_bytes.argtypes = [i32, i32, vp]
    L.lg_search_workspace_bytes.restype = sz
    L.lg_search.argtypes = [vp, vp, vp, i32, vp, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]
    L.lg_search_noalloc.argtypes = [vp, vp, vp, i32, vp, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    L.lg_search_noalloc_max_bytes.argtypes = []
    L.lg_search_noalloc_max_bytes.restype = sz
    L.lg_compact_unstable_workspace_bytes.argtypes = [i32, i32]
    L.lg_compact_unstable_workspace_bytes.restype = sz
    L.lg_compact_unstable.argtypes = [vp, vp, vp, i32, i32, i32, vp, vp, vp, sz, vp]
    L.lg_search_extend.argtypes = [vp, vp, vp, i32, vp, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp,
                                   vp, sz, vp]
    L.lg_realize.argtypes = [vp, vp, vp, vp, i32, vp, i32, vp, vp, i32, i32, vp, vp, i32, vp,
                             vp, vp, vp, vp, vp, vp]
    L.lg_serve_request_bytes.argtypes = [vp, vp]
    L.lg_serve_request_bytes.restype = C.c_uint64
    L.lg_serve_create.argtypes = [vp, vp]
    L.lg_serve_submit.argtypes = [vp, vp, vp]
    L.lg_serve_poll.argtypes = [vp, C.c_uint64, vp]
    L.lg_serve_wait.argtypes = [vp, C.c_uint64, C.c_double, vp]
    L.lg_serve_cancel.argtypes = [vp, C.c_uint64]
    L.lg_serve_stats.argtypes = [vp, vp]
    L.lg_serve_clock.argtypes = [vp]
    L.lg_serve_clock.restype = C.c_double
    L.lg_serve_destroy.argtypes = [vp]
    L.lg_place_exhaustive.argtypes = [vp, vp, vp, i32, i32, C.c_uint64, C.c_uint32, i64, vp, vp]
    L.lg_place_palm.argtypes = [vp, vp, vp, vp, i32, i32, C.c_float, C.c_float, C.c_uint64, C.c_uint32, i64, vp,
                                vp, vp]
    L.lg_concave_filter.argtypes = [vp, vp, vp, i32, C.c_float, i32, C.c_float, vp, vp, vp, vp, vp]
    L.lg_gather_points.argtypes = [vp, vp, i32, vp, i32, vp, vp, vp]
    L.lg_prop_num_params.restype = i64
    L.lg_prop_create.argtypes = [vp, vp, vp]
    L.lg_prop_release.argtypes = [vp]
    L.lg_prop_get_params.argtypes = [vp, vp]
    L.lg_prop_set_params.argtypes = [vp, vp]
    L.lg_prop_forward.argtypes = [vp, vp, i32, i32, vp, vp, vp, vp]
    L.lg_prop_backward.argtypes = [vp, vp, i32, i32, vp, vp, i32, vp, vp, vp]
    L.lg_prop_adam.argtypes = [vp, C.c_float, C.c_float, C.c_float, C.c_float, vp]
    L.lg_prop_train_step.argtypes = [vp, vp, i32, i32, vp, vp, i32, C.c_float, vp, vp]
    L.lg_prop_sample_mixture.argtypes = [vp, i32, C.c_uint64, C.c_float, C.c_float, C.c_float, vp, vp]
    L.lg_prop_sample.argtypes = [vp, vp, i32, i32, C.c_uint64, C.c_float, C.c_float, C.c_float, vp, vp]
    for fn in ("lg_build_field", "lg_field_import", "lg_field_export", "lg_field_info",
               "lg_field_release", "lg_query_domains", "lg_query_domains_cone", "lg_search", "lg_search_noalloc",
               "lg_compact_unstable", "lg_search_extend",
               "lg_realize", "lg_serve_create",
               "lg_serve_submit", "lg_serve_poll", "lg_serve_wait", "lg_serve_cancel", "lg_serve_stats",
               "lg_serve_destroy", "lg_place_exhaustive", "lg_place_palm", "lg_concave_filter", "lg_gather_points",
               "lg_query_domains_bounded", "lg_chunk_bounds", "lg_morton_order",
               "lg_prop_create", "lg_prop_release", "lg_prop_get_params",
               "lg_prop_set_params", "lg_prop_forward", "lg_prop_backward", "lg_prop_adam",
               "lg_prop_train_step", "lg_prop_sample_mixture", "lg_prop_sample"):
        getattr(L, fn).restype = i32
    return L


_lib = _load()

EXPORTED = ("lg_status_str", "lg_last_error", "lg_version", "lg_build_field", "lg_field_import",
            "lg_field_export", "lg_field_info", "lg_field_release", "lg_query_domains", "lg_query_domains_cone",
            "lg_query_domains_bounded", "lg_chunk_bounds", "lg_morton_order",
            "lg_search_workspace_bytes", "lg_search", "lg_search_noalloc", "lg_search_noalloc_max_bytes",
            "lg_compact_unstable_workspace_bytes", "lg_compact_unstable", "lg_search_extend",
            "lg_realize", "lg_serve_request_bytes",
            "lg_serve_create", "lg_serve_submit", "lg_serve_poll", "lg_serve_wait", "lg_serve_cancel",
            "lg_serve_stats", "lg_serve_clock", "lg_serve_destroy", "lg_place_exhaustive", "lg_place_palm",
            "lg_concave_filter",
            "lg_gather_points", "lg_prop_num_params",
            "lg_prop_create", "lg_prop_release", "lg_prop_get_params", "lg_prop_set_params",
            "lg_prop_forward", "lg_prop_backward", "lg_prop_adam", "lg_prop_train_step",
            "lg_prop_sample_mixture", "lg_prop_sample")


def lib():
    return _lib


def _check(st: int, where: str):
    if st != LG_OK:
        raise LgError(st, where, (_lib.lg_last_error() or b"").decode())


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return C.c_void_p(t.data_ptr())


def _hp(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _stream(stream) -> C.c_void_p:
    """hipStream_t of ``stream``; None means torch's current stream (the null
    stream before torch has touched the device)."""
    if stream is None:
        if not torch.cuda.is_initialized():
            return C.c_void_p(0)
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


class _HandKeep:
    def __init__(self, hand, palm=None):
        self.arrs = [np.ascontiguousarray(hand.joint_finger, np.int32),
                     np.ascontiguousarray(hand.joint_parent, np.int32),
                     np.ascontiguousarray(hand.joint_origin, np.float32),
                     np.ascontiguousarray(hand.joint_axis, np.float32),
                     np.ascontiguousarray(hand.capsule, np.float32),
                     np.ascontiguousarray(hand.limits, np.float32),
                     np.ascontiguousarray(hand.surf, np.float32)]
        a = self.arrs
        self.desc = HandDesc(int(hand.n_fingers), int(a[0].shape[0]), _hp(a[0]), _hp(a[1]), _hp(a[2]),
                             _hp(a[3]), _hp(a[4]), _hp(a[5]), int(a[6].shape[1]), _hp(a[6]), 0, None, 0, None)
        if palm is not None:
            ps = np.ascontiguousarray(palm.surf, np.float32)
            pc = np.ascontiguousarray(palm.caps, np.float32)
            self.arrs += [ps, pc]
            self.desc.n_palm_surf, self.desc.palm_surf = int(ps.shape[0]), _hp(ps)
            self.desc.n_palm_caps, self.desc.palm_caps = int(pc.shape[0]), _hp(pc)


def _field_params(fp, keep_witness: bool):
    gf = np.ascontiguousarray(fp.grid_frame, np.float32)
    return FieldParams(int(fp.samples), int(fp.seed) & 0xFFFFFFFFFFFFFFFF, int(fp.grid), float(fp.h),
                       int(fp.bins), _hp(gf), int(bool(keep_witness))), gf


class Field:
    """Owner of an ``lg_field`` handle (resident in HBM until released)."""

    def __init__(self, handle: C.c_void_p, hand):
        self.handle = handle
        self.n_fingers = int(hand.n_fingers)
        self.n_joints = int(hand.n_joints)

    def info(self) -> dict:
        inf = FieldInfo()
        _check(_lib.lg_field_info(self.handle, C.byref(inf)), "lg_field_info")
        return {k: getattr(inf, k) for k, _ in FieldInfo._fields_}

    def export(self, witness: bool = False):
        inf = self.info()
        L, G, B = inf["n_joints"], inf["grid"], inf["bins"]
        bits = np.zeros((L, G ** 3, B // 32), np.uint32)
        wit = np.zeros((L, G ** 3, B), np.int32) if witness else None
        _check(_lib.lg_field_export(self.handle, _hp(bits), None if wit is None else _hp(wit)),
               "lg_field_export")
        return bits, wit

    def release(self):
        if self.handle:
            _lib.lg_field_release(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass


# ---- the four calls of the hot path -----------------------------------------
def lg_build_field(hand, fp, keep_witness: bool = True, stream=None, palm=None) -> Field:
    """Build the contact field of ``hand``; ``palm`` (a static link with
    ``surf`` [S, 6] and ``caps`` [C, 7], base frame) is kept with it."""
    hk = _HandKeep(hand, palm)
    p, gf = _field_params(fp, keep_witness)
    out = C.c_void_p()
    _check(_lib.lg_build_field(C.byref(hk.desc), C.byref(p), _stream(stream), C.byref(out)),
           "lg_build_field")
    return Field(out, hand)


def lg_field_import(hand, fp, bits: np.ndarray, witness: Optional[np.ndarray] = None, palm=None) -> Field:
    hk = _HandKeep(hand, palm)
    p, gf = _field_params(fp, witness is not None)
    b = np.ascontiguousarray(bits, np.uint32)
    w = None if witness is None else np.ascontiguousarray(witness, np.int32)
    out = C.c_void_p()
    _check(_lib.lg_field_import(C.byref(hk.desc), C.byref(p), _hp(b), None if w is None else _hp(w),
                                C.byref(out)), "lg_field_import")
    return Field(out, hand)


def lg_query_domains(field: Field, pts: torch.Tensor, nrm: torch.Tensor, poses: torch.Tensor,
                     dom_bits: Optional[torch.Tensor] = None, dom_count: Optional[torch.Tensor] = None,
                     stream=None):
    """pts, nrm: [3, N] float32; poses: [P, 12] float32 (device tensors)."""
    N, P, F = int(pts.shape[1]), int(poses.shape[0]), field.n_fingers
    NW = (N + 31) // 32
    dev = pts.device
    if dom_bits is None:
        dom_bits = torch.empty((P, F, NW), dtype=torch.int32, device=dev)
    if dom_count is None:
        dom_count = torch.empty((P, F), dtype=torch.int32, device=dev)
    _check(_lib.lg_query_domains(field.handle, _ptr(pts), _ptr(nrm), N, _ptr(poses), P,
                                 _ptr(dom_bits), _ptr(dom_count), _stream(stream)), "lg_query_domains")
    return dom_bits, dom_count


def lg_query_domains_cone(field: Field, pts, nrm, poses, cos_hit: float, dom_bits=None, dom_count=None,
                          stream=None, bounds=None):
    """Cone (theta_hit) query; same shapes as lg_query_domains (``bounds``: optional chunk bounds)."""
    N, P, F = int(pts.shape[1]), int(poses.shape[0]), field.n_fingers
    NW = (N + 31) // 32
    dev = pts.device
    if dom_bits is None:
        dom_bits = torch.empty((P, F, NW), dtype=torch.int32, device=dev)
    if dom_count is None:
        dom_count = torch.empty((P, F), dtype=torch.int32, device=dev)
    _check(_lib.lg_query_domains_cone(field.handle, _ptr(pts), _ptr(nrm), N, _ptr(poses), P, _ptr(bounds),
                                      float(cos_hit), _ptr(dom_bits), _ptr(dom_count), _stream(stream)),
           "lg_query_domains_cone")
    return dom_bits, dom_count


def lg_chunk_bounds(pts: torch.Tensor, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """Bounding spheres [ceil(N/64), 4] (device) of the chunks of 64 consecutive points of SoA pts [3, N]."""
    N = int(pts.shape[1])
    if out is None:
        out = torch.empty((max(1, (N + 63) // 64), 4), dtype=torch.float32, device=pts.device)
    _check(_lib.lg_chunk_bounds(_ptr(pts), N, _ptr(out), _stream(stream)), "lg_chunk_bounds")
    return out


def lg_query_domains_bounded(field: Field, pts, nrm, poses, bounds, dom_bits=None, dom_count=None, stream=None):
    """lg_query_domains with chunk bounds (lg_chunk_bounds of the same points); identical outputs."""
    N, P, F = int(pts.shape[1]), int(poses.shape[0]), field.n_fingers
    NW = (N + 31) // 32
    dev = pts.device
    if dom_bits is None:
        dom_bits = torch.empty((P, F, NW), dtype=torch.int32, device=dev)
    if dom_count is None:
        dom_count = torch.empty((P, F), dtype=torch.int32, device=dev)
    _check(_lib.lg_query_domains_bounded(field.handle, _ptr(pts), _ptr(nrm), N, _ptr(poses), P, _ptr(bounds),
                                         _ptr(dom_bits), _ptr(dom_count), _stream(stream)),
           "lg_query_domains_bounded")
    return dom_bits, dom_count


def lg_morton_order(pts_host: np.ndarray) -> np.ndarray:
    """Morton permutation (int32 [N]) of host points [N, 3]."""
    p = np.ascontiguousarray(pts_host, np.float32)
    perm = np.zeros(p.shape[0], np.int32)
    _check(_lib.lg_morton_order(_hp(p), int(p.shape[0]), _hp(perm)), "lg_morton_order")
    return perm


def search_params(sp, max_pivots: int = 1000) -> SearchParams:
    return SearchParams(int(sp.draws), int(sp.k), int(sp.m_edges), int(max_pivots), float(sp.mu),
                        float(sp.eps), float(sp.moment_scale), int(sp.seed) & 0xFFFFFFFFFFFFFFFF,
                        int(sp.request_id), int(sp.pose_offset), int(getattr(sp, "opt_outer", 0)),
                        int(getattr(sp, "opt_inner", 8)), float(getattr(sp, "opt_sigma", 0.004)))


class SearchBuffers:
    """Device outputs + workspace of lg_search for P poses (reusable)."""

    def __init__(self, n_poses: int, sp, device, max_pivots: int = 1000, n_points: int = 0):
        self.p = search_params(sp, max_pivots)
        P, D, k = n_poses, int(sp.draws), int(sp.k)
        self.set_pt = torch.empty((P, D, k), dtype=torch.int32, device=device)
        self.set_link = torch.empty((P, D, k), dtype=torch.int8, device=device)
        self.verdict = torch.empty((P, D), dtype=torch.uint8, device=device)
        self.tstar = torch.empty((P, D), dtype=torch.float64, device=device)
        self.acc_list = torch.empty((P * D,), dtype=torch.int32, device=device)
        self.n_acc = torch.zeros((1,), dtype=torch.int32, device=device)
        nb = int(_lib.lg_search_workspace_bytes(int(n_points), P, C.byref(self.p)))
        self.workspace = torch.empty((nb,), dtype=torch.uint8, device=device)


def lg_search(field: Field, pts, nrm, poses, dom_bits, dom_count, sp, bufs: Optional[SearchBuffers] = None,
              max_pivots: int = 1000, stream=None, palm_pt: Optional[torch.Tensor] = None) -> SearchBuffers:
    """``palm_pt`` (device int32 [P], from lg_place_palm): each pose's fixed palm contact."""
    N, P = int(pts.shape[1]), int(poses.shape[0])
    if bufs is None:
        bufs = SearchBuffers(P, sp, pts.device, max_pivots, n_points=N)
    bufs.p.palm_pt = None if palm_pt is None else palm_pt.data_ptr()
    bufs.palm_pt = palm_pt          # the struct holds only its address
    _check(_lib.lg_search(field.handle, _ptr(pts), _ptr(nrm), N, _ptr(poses), P, _ptr(dom_bits),
                          _ptr(dom_count), C.byref(bufs.p), _ptr(bufs.set_pt), _ptr(bufs.set_link),
                          _ptr(bufs.verdict), _ptr(bufs.tstar), _ptr(bufs.acc_list), _ptr(bufs.n_acc),
                          _ptr(bufs.workspace), bufs.workspace.numel(), _stream(stream)), "lg_search")
    return bufs


def lg_search_noalloc(field: Field, pts, nrm, poses, dom_bits, dom_count, sp, bufs: SearchBuffers,
                      max_pivots: int = 1000, stream=None, palm_pt: Optional[torch.Tensor] = None) -> SearchBuffers:
    """lg_search on the library's static device scratch (no workspace argument,
    nothing allocated by the call; ``bufs`` holds the caller's outputs)."""
    N, P = int(pts.shape[1]), int(poses.shape[0])
    bufs.p = search_params(sp, max_pivots)
    bufs.p.palm_pt = None if palm_pt is None else palm_pt.data_ptr()
    bufs.palm_pt = palm_pt
    _check(_lib.lg_search_noalloc(field.handle, _ptr(pts), _ptr(nrm), N, _ptr(poses), P, _ptr(dom_bits),
                                  _ptr(dom_count), C.byref(bufs.p), _ptr(bufs.set_pt), _ptr(bufs.set_link),
                                  _ptr(bufs.verdict), _ptr(bufs.tstar), _ptr(bufs.acc_list), _ptr(bufs.n_acc),
                                  _stream(stream)), "lg_search_noalloc")
    return bufs


def lg_compact_unstable(bufs: SearchBuffers, stream=None, out=None):
    """Increasing ids of the sets of ``bufs`` (a search) with a whole draw and
    verdict 0; returns (list [P*D] int32, n_list [1] int32, workspace) on the
    device (``out``: the same triple from an earlier call, reused)."""
    P, D, k = (int(x) for x in bufs.set_pt.shape)
    dev = bufs.set_pt.device
    nb = int(_lib.lg_compact_unstable_workspace_bytes(P, D))
    if out is None:
        out = (torch.empty((P * D,), dtype=torch.int32, device=dev), torch.zeros((1,), dtype=torch.int32, device=dev),
               torch.empty((nb,), dtype=torch.uint8, device=dev))
    lst, n, ws = out
    _check(_lib.lg_compact_unstable(_ptr(bufs.set_pt), _ptr(bufs.set_link), _ptr(bufs.verdict), P, D, k, _ptr(lst),
                                    _ptr(n), _ptr(ws), nb, _stream(stream)), "lg_compact_unstable")
    return out


class ExtendBuffers:
    """Device outputs + workspace of lg_search_extend for P poses."""

    def __init__(self, n_poses: int, sp, k_add: int, device, max_pivots: int = 1000, n_points: int = 0):
        P, D, k2 = n_poses, int(sp.draws), int(sp.k) + int(k_add)
        self.set_pt = torch.empty((P, D, k2), dtype=torch.int32, device=device)
        self.set_link = torch.empty((P, D, k2), dtype=torch.int8, device=device)
        self.verdict = torch.empty((P, D), dtype=torch.uint8, device=device)
        self.tstar = torch.empty((P, D), dtype=torch.float64, device=device)
        self.acc_list = torch.empty((P * D,), dtype=torch.int32, device=device)
        self.n_acc = torch.zeros((1,), dtype=torch.int32, device=device)
        p2 = search_params(sp, max_pivots)
        p2.k = k2
        p2.opt_outer = 0
        nb = int(_lib.lg_search_workspace_bytes(int(n_points), P, C.byref(p2)))
        self.workspace = torch.empty((nb,), dtype=torch.uint8, device=device)


def lg_search_extend(field: Field, pts, nrm, poses, dom_bits, dom_count, sp, round1: SearchBuffers, k_add: int,
                     request_id: int = 0, set_list=None, list_n=None, list_ok=None,
                     bufs: Optional[ExtendBuffers] = None, max_pivots: int = 1000, stream=None) -> ExtendBuffers:
    """Second contact round on the unused fingers of ``round1``'s sets (search
    parameters ``sp``); ``set_list``/``list_n``/``list_ok``: device arrays
    choosing the sets (default: every unstable set with a whole draw)."""
    N, P = int(pts.shape[1]), int(poses.shape[0])
    if bufs is None:
        bufs = ExtendBuffers(P, sp, k_add, pts.device, max_pivots, n_points=N)
    p1 = search_params(sp, max_pivots)
    ep = ExtendParams(int(k_add), int(request_id), None if set_list is None else set_list.data_ptr(),
                      None if list_n is None else list_n.data_ptr(), None if list_ok is None else list_ok.data_ptr())
    _check(_lib.lg_search_extend(field.handle, _ptr(pts), _ptr(nrm), N, _ptr(poses), P, _ptr(dom_bits),
                                 _ptr(dom_count), C.byref(p1), _ptr(round1.set_pt), _ptr(round1.set_link),
                                 _ptr(round1.verdict), C.byref(ep), _ptr(bufs.set_pt), _ptr(bufs.set_link),
                                 _ptr(bufs.verdict), _ptr(bufs.tstar), _ptr(bufs.acc_list), _ptr(bufs.n_acc),
                                 _ptr(bufs.workspace), bufs.workspace.numel(), _stream(stream)), "lg_search_extend")
    return bufs


def ik_params(ik, sp=None) -> IkParams:
    """Realize parameters; the random joints of fingers without contact are keyed
    by the search parameters ``sp`` (seed, request_id, pose_offset)."""
    seed, rid, off = (0, 0, 0) if sp is None else (int(sp.seed) & 0xFFFFFFFFFFFFFFFF, int(sp.request_id),
                                                    int(sp.pose_offset))
    return IkParams(int(ik.iters), int(ik.phase1), float(ik.lam), float(ik.beta), float(ik.tol_pos),
                    float(ik.tol_ang), float(ik.margin), int(getattr(ik, "self_collision", 0)), seed, rid, off)


def sdf_struct(sdf_host, values_dev: torch.Tensor) -> Sdf:
    o = np.asarray(sdf_host.origin, np.float32)
    return Sdf((C.c_float * 3)(*[float(x) for x in o]), float(sdf_host.h), int(sdf_host.dims),
               C.c_void_p(values_dev.data_ptr()))


class RealizeBuffers:
    def __init__(self, max_acc: int, n_joints: int, k: int, device):
        self.q = torch.empty((max_acc, n_joints), dtype=torch.float32, device=device)
        self.contact_err = torch.empty((max_acc, k), dtype=torch.float32, device=device)
        self.contact_ang = torch.empty((max_acc, k), dtype=torch.float32, device=device)
        self.depth = torch.empty((max_acc,), dtype=torch.float32, device=device)
        self.valid = torch.empty((max_acc,), dtype=torch.uint8, device=device)


def lg_realize(field: Field, sdf: Sdf, pts, nrm, poses, set_pt, set_link, k: int, draws: int, acc_list,
               n_acc_dev, max_acc: int, ik, bufs: Optional[RealizeBuffers] = None, stream=None, sp=None):
    N, P = int(pts.shape[1]), int(poses.shape[0])
    if bufs is None:
        bufs = RealizeBuffers(max_acc, field.n_joints, k, pts.device)
    ikp = ik_params(ik, sp)
    _check(_lib.lg_realize(field.handle, C.byref(sdf), _ptr(pts), _ptr(nrm), N, _ptr(poses), P,
                           _ptr(set_pt), _ptr(set_link), int(k), int(draws), _ptr(acc_list), _ptr(n_acc_dev),
                           int(max_acc), C.byref(ikp), _ptr(bufs.q), _ptr(bufs.contact_err),
                           _ptr(bufs.contact_ang), _ptr(bufs.depth), _ptr(bufs.valid), _stream(stream)),
           "lg_realize")
    return bufs


def version() -> str:
    return _lib.lg_version().decode()


def lg_place_palm(field: Field, sdf: Sdf, pts: torch.Tensor, nrm: torch.Tensor, poses: torch.Tensor, prob: float,
                  margin: float, seed: int, request_id: int = 0, pose_offset: int = 0,
                  palm_pt: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """Static-link placements in place over device poses [P, 12]; returns palm_pt [P] int32."""
    N, P = int(pts.shape[1]), int(poses.shape[0])
    if palm_pt is None:
        palm_pt = torch.empty((P,), dtype=torch.int32, device=pts.device)
    _check(_lib.lg_place_palm(field.handle, C.byref(sdf), _ptr(pts), _ptr(nrm), N, P, float(prob), float(margin),
                              int(seed) & 0xFFFFFFFFFFFFFFFF, int(request_id), int(pose_offset), _ptr(poses),
                              _ptr(palm_pt), _stream(stream)), "lg_place_palm")
    return palm_pt


def lg_place_exhaustive(field: Field, pts: torch.Tensor, nrm: torch.Tensor, n_poses: int, seed: int,
                        request_id: int = 0, pose_offset: int = 0, out: Optional[torch.Tensor] = None,
                        stream=None) -> torch.Tensor:
    """Exhaustive-placement poses [n_poses, 12] (device) for SoA points/normals [3, N]."""
    N = int(pts.shape[1])
    if out is None:
        out = torch.empty((n_poses, 12), dtype=torch.float32, device=pts.device)
    _check(_lib.lg_place_exhaustive(field.handle, _ptr(pts), _ptr(nrm), N, int(n_poses),
                                    int(seed) & 0xFFFFFFFFFFFFFFFF, int(request_id), int(pose_offset),
                                    _ptr(out), _stream(stream)), "lg_place_exhaustive")
    return out


class ConcaveResult:
    """Device outputs of lg_concave_filter for N points."""

    def __init__(self, n_points: int, device):
        n = max(1, n_points)
        self.depth = torch.empty((n,), dtype=torch.float32, device=device)
        self.keep = torch.empty((n,), dtype=torch.uint8, device=device)
        self.kept_idx = torch.empty((n,), dtype=torch.int32, device=device)
        self.n_kept = torch.zeros((1,), dtype=torch.int32, device=device)


def lg_concave_filter(sdf: Sdf, pts: torch.Tensor, nrm: torch.Tensor, box_edge: float = 0.008, lattice: int = 4,
                      max_depth: float = 0.001, out: Optional[ConcaveResult] = None, stream=None) -> ConcaveResult:
    """Sec. 5.2 concave-point removal over SoA points/normals [3, N] (device)."""
    N = int(pts.shape[1])
    if out is None:
        out = ConcaveResult(N, pts.device)
    _check(_lib.lg_concave_filter(C.byref(sdf), _ptr(pts), _ptr(nrm), N, float(box_edge), int(lattice),
                                  float(max_depth), _ptr(out.depth), _ptr(out.keep), _ptr(out.kept_idx),
                                  _ptr(out.n_kept), _stream(stream)), "lg_concave_filter")
    return out


def lg_gather_points(pts: torch.Tensor, nrm: torch.Tensor, idx: torch.Tensor, n_out: int, stream=None):
    """SoA [3, n_out] copies of the columns idx[:n_out] of pts/nrm [3, N] (device)."""
    N = int(pts.shape[1])
    po = torch.empty((3, n_out), dtype=torch.float32, device=pts.device)
    no = torch.empty((3, n_out), dtype=torch.float32, device=pts.device)
    _check(_lib.lg_gather_points(_ptr(pts), _ptr(nrm), N, _ptr(idx), int(n_out), _ptr(po), _ptr(no),
                                 _stream(stream)), "lg_gather_points")
    return po, no


# ---- serving -----------------------------------------------------------------
def result_dict(r: Result) -> dict:
    return {k: getattr(r, k) for k, _ in Result._fields_}


class Server:
    """Continuous-batching server over resident fields (see ``lg_serve_*``).
    ``batched``: run the chunks of all idle requests as one launch per stage
    over a per-chunk descriptor table (else one stream per request)."""

    def __init__(self, budget_bytes: int, max_active: int = 8, chunk_poses: int = 4096, batched: bool = True,
                 batch_slots: int = 0):
        self.params = ServerParams(int(budget_bytes), int(max_active), int(chunk_poses), int(bool(batched)),
                                   int(batch_slots))
        h = C.c_void_p()
        _check(_lib.lg_serve_create(C.byref(self.params), C.byref(h)), "lg_serve_create")
        self.handle = h
        self._keep = {}

    def make_request(self, field: Field, pts: np.ndarray, nrm: np.ndarray, poses: np.ndarray, sp,
                     request_id: int, ik=None, sdf=None, max_pivots: int = 1000):
        pts = np.ascontiguousarray(pts, np.float32)
        nrm = np.ascontiguousarray(nrm, np.float32)
        poses = np.ascontiguousarray(poses, np.float32)
        keep = [pts, nrm, poses]
        req = Request()
        req.field = field.handle
        req.pts, req.nrm, req.poses = _hp(pts), _hp(nrm), _hp(poses)
        req.n_points, req.n_poses = int(pts.shape[0]), int(poses.shape[0])
        req.search = search_params(sp, max_pivots)
        req.request_id = int(request_id)
        if ik is not None:
            vals = np.ascontiguousarray(sdf.values, np.float32)
            keep.append(vals)
            req.realize = 1
            req.ik = ik_params(ik)
            req.sdf_values = _hp(vals)
            req.sdf_origin = (C.c_float * 3)(*[float(x) for x in np.asarray(sdf.origin, np.float32)])
            req.sdf_h = float(sdf.h)
            req.sdf_dims = int(sdf.dims)
        return req, keep

    def request_bytes(self, req: Request) -> int:
        return int(_lib.lg_serve_request_bytes(C.byref(self.params), C.byref(req)))

    def submit(self, req: Request) -> int:
        t = C.c_uint64()
        _check(_lib.lg_serve_submit(self.handle, C.byref(req), C.byref(t)), "lg_serve_submit")
        return int(t.value)

    def poll(self, ticket: int) -> dict:
        r = Result()
        _check(_lib.lg_serve_poll(self.handle, int(ticket), C.byref(r)), "lg_serve_poll")
        return result_dict(r)

    def wait(self, ticket: int, timeout_s: float = 60.0) -> dict:
        r = Result()
        _check(_lib.lg_serve_wait(self.handle, int(ticket), float(timeout_s), C.byref(r)), "lg_serve_wait")
        return result_dict(r)

    def cancel(self, ticket: int):
        _check(_lib.lg_serve_cancel(self.handle, int(ticket)), "lg_serve_cancel")

    def stats(self) -> dict:
        st = ServerStats()
        _check(_lib.lg_serve_stats(self.handle, C.byref(st)), "lg_serve_stats")
        return {k: getattr(st, k) for k, _ in ServerStats._fields_}

    def clock(self) -> float:
        return float(_lib.lg_serve_clock(self.handle))

    def destroy(self):
        if self.handle:
            _lib.lg_serve_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def mix64(z: int) -> int:
    """splitmix64 finaliser used for the order-independent accepted-set hash."""
    m = (1 << 64) - 1
    z = (z + 0x9E3779B97F4A7C15) & m
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & m
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & m
    return z ^ (z >> 31)


def accepted_hash(request_id: int, acc_ids) -> int:
    """Hash the server reports for accepted set ids (pose * D + draw)."""
    h = 0
    for i in acc_ids:
        h = (h + mix64(((int(request_id) << 40) ^ int(i)) & ((1 << 64) - 1))) & ((1 << 64) - 1)
    return h


# ---- learned palm-pose proposer ---------------------------------------------
PROP_OUT = 152
PROP_FEAT = 256


class PropParams(C.Structure):
    _fields_ = [("max_batch", C.c_int32), ("max_points", C.c_int32), ("max_targets", C.c_int32),
                ("seed", C.c_uint64)]


def lg_prop_num_params() -> int:
    return int(_lib.lg_prop_num_params())


class Proposer:
    """A proposer owned by the library (see ``lg_prop_*``).  Inputs ``x`` are
    device float32 tensors [B][Np][6] of (p in m, unit normal)."""

    def __init__(self, max_batch: int = 64, max_points: int = 2048, max_targets: int = 1 << 16,
                 seed: int = 0, stream=None):
        self.params = PropParams(int(max_batch), int(max_points), int(max_targets), int(seed))
        h = C.c_void_p()
        _check(_lib.lg_prop_create(C.byref(self.params), _stream(stream), C.byref(h)), "lg_prop_create")
        self.handle = h
        self.n_params = lg_prop_num_params()

    def get_params(self) -> np.ndarray:
        out = np.zeros(self.n_params, np.float32)
        _check(_lib.lg_prop_get_params(self.handle, _hp(out)), "lg_prop_get_params")
        return out

    def set_params(self, flat) -> None:
        a = np.ascontiguousarray(flat, np.float32)
        if a.size != self.n_params:
            raise ValueError("parameter vector has the wrong length")
        _check(_lib.lg_prop_set_params(self.handle, _hp(a)), "lg_prop_set_params")

    def forward(self, x: torch.Tensor, stream=None) -> dict:
        B, Np = int(x.shape[0]), int(x.shape[1])
        dev = x.device
        out = torch.empty((B, PROP_OUT), dtype=torch.float32, device=dev)
        feat = torch.empty((B, PROP_FEAT), dtype=torch.float32, device=dev)
        arg = torch.empty((B, PROP_FEAT), dtype=torch.int32, device=dev)
        _check(_lib.lg_prop_forward(self.handle, _ptr(x), B, Np, _ptr(out), _ptr(feat), _ptr(arg),
                                    _stream(stream)), "lg_prop_forward")
        return {"out": out, "feat": feat, "arg": arg}

    def backward(self, x: torch.Tensor, targets: torch.Tensor, offsets: torch.Tensor, stream=None):
        B, Np = int(x.shape[0]), int(x.shape[1])
        loss = torch.empty(1, dtype=torch.float32, device=x.device)
        grad = torch.empty(self.n_params, dtype=torch.float32, device=x.device)
        _check(_lib.lg_prop_backward(self.handle, _ptr(x), B, Np, _ptr(targets), _ptr(offsets),
                                     int(targets.shape[0]), _ptr(loss), _ptr(grad), _stream(stream)),
               "lg_prop_backward")
        return loss, grad

    def adam(self, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8, stream=None):
        _check(_lib.lg_prop_adam(self.handle, float(lr), float(beta1), float(beta2), float(eps),
                                 _stream(stream)), "lg_prop_adam")

    def train_step(self, x: torch.Tensor, targets: torch.Tensor, offsets: torch.Tensor, lr: float,
                   loss: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        B, Np = int(x.shape[0]), int(x.shape[1])
        if loss is None:
            loss = torch.empty(1, dtype=torch.float32, device=x.device)
        _check(_lib.lg_prop_train_step(self.handle, _ptr(x), B, Np, _ptr(targets), _ptr(offsets),
                                       int(targets.shape[0]), float(lr), _ptr(loss), _stream(stream)),
               "lg_prop_train_step")
        return loss

    def sample(self, x: torch.Tensor, n_poses: int, seed: int, uniform_frac: float,
               d_lo: float = 0.08, d_hi: float = 0.12, out: Optional[torch.Tensor] = None,
               stream=None) -> torch.Tensor:
        Np = int(x.shape[-2])
        if out is None:
            out = torch.empty((n_poses, 12), dtype=torch.float32, device=x.device)
        _check(_lib.lg_prop_sample(self.handle, _ptr(x), Np, int(n_poses), int(seed), float(uniform_frac),
                                   float(d_lo), float(d_hi), _ptr(out), _stream(stream)), "lg_prop_sample")
        return out

    def release(self):
        if self.handle:
            _lib.lg_prop_release(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass


def lg_prop_sample_mixture(mix: torch.Tensor, n_poses: int, seed: int, uniform_frac: float,
                           d_lo: float = 0.08, d_hi: float = 0.12, stream=None) -> torch.Tensor:
    out = torch.empty((n_poses, 12), dtype=torch.float32, device=mix.device)
    _check(_lib.lg_prop_sample_mixture(_ptr(mix), int(n_poses), int(seed), float(uniform_frac), float(d_lo),
                                       float(d_hi), _ptr(out), _stream(stream)), "lg_prop_sample_mixture")
    return out
