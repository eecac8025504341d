"""One pass of the hot path over a batch of palm poses, with every input and
buffer resident in device memory: lg_query_domains -> lg_search ->
lg_realize (Fig. 6 pipeline: placement given, domain generation, contact
sets + criterion, kinematics + collision filtering)."""
from __future__ import annotations

from typing import Optional

import numpy as np
import torch

from . import lg


class Pipeline:
    """Holds the object, poses and all per-step buffers of one workload.

    ``step()`` enqueues the whole path on ``stream`` and returns without
    synchronising; ``valid_count()`` synchronises and reads the result."""

    def __init__(self, field: lg.Field, pts: np.ndarray, nrm: np.ndarray, poses: np.ndarray, sp,
                 ik=None, sdf=None, device: str = "cuda", max_pivots: int = 1000, cos_hit=None, palm_pt=None,
                 extend_k: int = 0, extend_request: int = 7):
        self.field = field
        self.palm_pt = palm_pt      # device int32 [P] of lg_place_palm, or None (no static-link contacts)
        self.cos_hit = cos_hit      # None: nearest-bin query; else the cone (theta_hit) query
        self.dev = torch.device(device)
        self.pts = torch.from_numpy(np.ascontiguousarray(np.asarray(pts, np.float32).T)).to(self.dev)
        self.nrm = torch.from_numpy(np.ascontiguousarray(np.asarray(nrm, np.float32).T)).to(self.dev)
        if isinstance(poses, torch.Tensor):       # already on the device (e.g. proposer output)
            self.poses = poses.to(self.dev, torch.float32).contiguous()
        else:
            self.poses = torch.from_numpy(np.ascontiguousarray(poses, np.float32)).to(self.dev)
        self.N, self.P = int(self.pts.shape[1]), int(self.poses.shape[0])
        # bounding spheres of the object's 64-point chunks (once per object): the
        # query skips (chunk, finger) pairs that cannot reach the finger's window
        self.bounds = lg.lg_chunk_bounds(self.pts) if self.N > 0 else None
        self.sp = sp
        F = field.n_fingers
        NW = (self.N + 31) // 32
        self.dom_bits = torch.empty((self.P, F, NW), dtype=torch.int32, device=self.dev)
        self.dom_count = torch.empty((self.P, F), dtype=torch.int32, device=self.dev)
        self.sbuf = lg.SearchBuffers(self.P, sp, self.dev, max_pivots, n_points=self.N)
        self.ik = ik
        self.rbuf = None
        if ik is not None:
            if sdf is None:
                raise ValueError("realize needs an SDF")
            self.sdf_vals = torch.from_numpy(np.ascontiguousarray(sdf.values, np.float32)).to(self.dev)
            self.sdf = lg.sdf_struct(sdf, self.sdf_vals)
            self.max_acc = self.P * int(sp.draws)
            self.rbuf = lg.RealizeBuffers(self.max_acc, field.n_joints, int(sp.k), self.dev)
        # the general form (Sec. 5.3, 5.6): unstable round-1 sets that realise
        # collision-free get extend_k more contacts on unused fingers
        self.extend_k = int(extend_k)
        self.extend_request = int(extend_request)
        if self.extend_k > 0:
            if ik is None:
                raise ValueError("the second contact round needs realize (ik, sdf)")
            self.unstable = None
            self.rbuf_rej = lg.RealizeBuffers(self.max_acc, field.n_joints, int(sp.k), self.dev)
            self.ebuf = lg.ExtendBuffers(self.P, sp, self.extend_k, self.dev, max_pivots, n_points=self.N)
            self.rbuf2 = lg.RealizeBuffers(self.max_acc, field.n_joints, int(sp.k) + self.extend_k, self.dev)
            import dataclasses
            self.sp2 = dataclasses.replace(sp, k=int(sp.k) + self.extend_k)

    def query(self, stream=None):
        if self.cos_hit is None:
            lg.lg_query_domains_bounded(self.field, self.pts, self.nrm, self.poses, self.bounds, self.dom_bits,
                                        self.dom_count, stream=stream)
        else:
            lg.lg_query_domains_cone(self.field, self.pts, self.nrm, self.poses, self.cos_hit, self.dom_bits,
                                     self.dom_count, stream=stream, bounds=self.bounds)

    def search(self, stream=None, request_id=None):
        """Draws + verdicts on the current domains; another request_id resamples
        the same domains (multi-pass reuse of a query)."""
        if request_id is not None:
            self.sbuf.p.request_id = int(request_id)
        lg.lg_search(self.field, self.pts, self.nrm, self.poses, self.dom_bits, self.dom_count, self.sp,
                     bufs=self.sbuf, stream=stream, palm_pt=self.palm_pt)

    def realize(self, stream=None):
        if self.ik is None:
            return
        b = self.sbuf
        lg.lg_realize(self.field, self.sdf, self.pts, self.nrm, self.poses, b.set_pt, b.set_link,
                      int(self.sp.k), int(self.sp.draws), b.acc_list, b.n_acc, self.max_acc, self.ik,
                      bufs=self.rbuf, stream=stream, sp=b.p)

    def extend(self, stream=None):
        """Second contact round: list the unstable sets, realise them with k
        contacts, extend those that realise collision-free, realise the
        accepted extended sets."""
        b, k = self.sbuf, int(self.sp.k)
        self.unstable = lg.lg_compact_unstable(b, stream=stream, out=self.unstable)
        lst, n, _ = self.unstable
        lg.lg_realize(self.field, self.sdf, self.pts, self.nrm, self.poses, b.set_pt, b.set_link, k,
                      int(self.sp.draws), lst, n, self.max_acc, self.ik, bufs=self.rbuf_rej, stream=stream, sp=b.p)
        lg.lg_search_extend(self.field, self.pts, self.nrm, self.poses, self.dom_bits, self.dom_count, self.sp, b,
                            self.extend_k, request_id=self.extend_request, set_list=lst, list_n=n,
                            list_ok=self.rbuf_rej.valid, bufs=self.ebuf, stream=stream)
        e = self.ebuf
        lg.lg_realize(self.field, self.sdf, self.pts, self.nrm, self.poses, e.set_pt, e.set_link,
                      int(self.sp2.k), int(self.sp.draws), e.acc_list, e.n_acc, self.max_acc, self.ik,
                      bufs=self.rbuf2, stream=stream, sp=b.p)

    def step(self, stream=None):
        self.query(stream)
        self.search(stream)
        self.realize(stream)
        if self.extend_k > 0:
            self.extend(stream)

    def n_acc(self) -> int:
        return int(self.sbuf.n_acc.item())

    def valid_sets(self) -> torch.Tensor:
        """Global set ids (g * D + d) of the valid grasps of the last step."""
        n = self.n_acc()
        ids = self.sbuf.acc_list[:n]
        if self.ik is None:
            return ids
        return ids[self.rbuf.valid[:n] != 0]

    def valid_count(self) -> int:
        """Valid grasps of the last step: accepted sets that pass IK and
        penetration (with realize), else accepted (verdict) sets; with the
        second contact round, plus its accepted extended sets that pass."""
        n = self.n_acc()
        if self.ik is None:
            return n
        v = int(self.rbuf.valid[:n].sum().item())
        if self.extend_k > 0:
            n2 = int(self.ebuf.n_acc.item())
            v += int(self.rbuf2.valid[:n2].sum().item())
        return v
