"""Benchmark of the Contact-Field hot path on one MI355X.

A step is one pass of the whole path over one batch of palm poses with the
field prebuilt and resident (Fig. 6: the field is built once per hand and
cached): contact-domain query -> draws + force-closure verdicts + compaction
-> DLS IK + penetration.  Inputs are seeded synthetic workloads (see
``synth``), resident in HBM before the timed region.

Prints ONE JSON line: valid grasps per second (whole job), the query kernel's
roofline (algorithmic bytes / measured kernel time vs 8 TB/s HBM), per-stage
times, and the FP64 CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "valid grasps/sec per object (1 GPU); field-query HBM GB/s; p50/p99 latency"
HBM_PEAK_GBPS = 8000.0
FP32_PEAK_TFLOPS = 157.3

DESCR = {
    "c1": "3-finger 9-DOF hand, sphere R=40mm N=2048, P=256, D=16, k=3, field 32^3@4mm B=32 S=8192",
    "c2": "4-finger 16-DOF hand, superquadric N=16384, P=16384, D=32, k=4, field 64^3@3mm B=64 S=262144",
    "c3": "5-finger 22-DOF hand, tool union N=65536, P=65536, D=64, k=5, field 64^3@3mm B=64 S=262144, "
          "IK 10 it lambda=1e-2, SDF 64^3",
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c3", choices=["c1", "c2", "c3"])
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cpu-poses", type=int, default=0, help="poses of the CPU-oracle sample (0 = auto)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve-rate", type=float, default=20.0, help="Poisson arrival rate of the serving run (req/s)")
    ap.add_argument("--serve-rates", default="5,20,50,100,400", help="serve mode: comma-separated arrival rates")
    ap.add_argument("--serve-seconds", type=float, default=6.0, help="arrival window of the serving run (s)")
    ap.add_argument("--serve-requests", type=int, default=0,
                    help="serve mode: exactly this many requests per rate (0: Poisson count over --serve-seconds)")
    ap.add_argument("--serve-modes", default="batched",
                    help="serve mode: comma-separated server modes, 'batched' (descriptor-table launches) "
                         "and/or 'streams' (one stream per request)")
    ap.add_argument("--serve-alone", type=int, default=40, help="requests of each stream re-run one at a time")
    ap.add_argument("--serve-slots", type=int, default=0, help="batched server: batches in flight (0: default)")
    ap.add_argument("--serve-chunk", type=int, default=4096, help="server: poses per chunk")
    ap.add_argument("--serve-active", type=int, default=8, help="server: requests admitted at once")
    ap.add_argument("--serve-mix", default="c4", choices=["c4", "small"],
                    help="request mix: c4 (N log-U[2k,64k], poses log-U[1k,64k]) or small "
                         "(N log-U[2k,4k], poses log-U[1k,2k])")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--opt-outer", type=int, default=0,
                    help="rounds of contact-point optimisation (Alg. 2) before the verdicts; 0 = the plain method")
    ap.add_argument("--opt-inner", type=int, default=8)
    ap.add_argument("--self-collision", action="store_true",
                    help="also reject grasps whose links of different fingers penetrate")
    ap.add_argument("--opt-sigma", type=float, default=0.004)
    ap.add_argument("--train-objects", type=int, default=2000, help="proposer: training objects (seeds 0..n-1)")
    ap.add_argument("--eval-objects", type=int, default=200, help="proposer: held-out objects (seeds 100000..)")
    ap.add_argument("--epochs", type=int, default=60, help="proposer: training epochs")
    ap.add_argument("--passes", type=int, default=8, help="multipass: searches per query")
    ap.add_argument("--cone-deg", type=float, default=0.0,
                    help="use the cone (theta_hit) query with this half-angle in degrees; 0 = nearest bin")
    ap.add_argument("--k", type=int, default=0,
                    help="contacts per set (0 = one per finger); below the finger count, k fingers are drawn "
                         "per set and the others take random joint values")
    ap.add_argument("--extend", type=int, default=0,
                    help="second contact round (the general form, Sec. 5.3/5.6): unstable sets that realise "
                         "collision-free get this many more contacts on unused fingers (needs --k below the "
                         "finger count)")
    ap.add_argument("--concave-filter", action="store_true",
                    help="drop the object's concave points first (8 mm box, 1 mm depth); the steps use the rest")
    ap.add_argument("--palm-prob", type=float, default=0.0,
                    help="probability of a static-link (palm) placement per pose (Sec. 5.1); 0 = none")
    ap.add_argument("--placement", default="canonical", choices=["canonical", "exhaustive"],
                    help="palm poses: canonical (random pose above the palm) or exhaustive (an object point "
                         "on a random contact vector of the field)")
    ap.add_argument("--mode", default="full",
                    choices=["full", "query", "search", "serve", "proposer", "encoder", "multipass"],
                    help="query / search: only the field build and --steps launches of that stage "
                         "(query mode adds a 1 GiB device copy); for hardware-counter runs, no JSON")
    return ap.parse_args()


def in_window_lookups(torch, pipe, w) -> list:
    """Exact number, per finger, of (pose, point) pairs whose point lies
    inside the finger's window (the links of a finger share it), counted on
    the device in float32 (the query's precision)."""
    gf = torch.from_numpy(np.asarray(w.field.grid_frame, np.float32).reshape(-1, 3, 4)).cuda()
    Rg, og = gf[:, :, :3], gf[:, :, 3]
    G, h = w.field.grid, float(np.float32(w.field.h))
    pts = pipe.pts  # [3, N]
    total = torch.zeros(gf.shape[0], dtype=torch.int64, device="cuda")
    chunk = max(1, int(2 ** 26 // (pts.shape[1] * gf.shape[0])))
    for g0 in range(0, pipe.P, chunk):
        P = pipe.poses[g0:g0 + chunk].reshape(-1, 3, 4)
        x = P[:, :, :3] @ pts + P[:, :, 3:4]                                # [p, 3, N]
        u = torch.einsum("fab,pan->pfbn", Rg, x) - torch.einsum("fab,fa->fb", Rg, og)[None, :, :, None]
        u = torch.floor(u / h)
        inside = ((u >= 0) & (u < G)).all(dim=2)                          # [p, f, N]
        total += inside.sum(dim=(0, 2))
    return [int(x) for x in total.cpu()]


def query_traffic():
    """HBM bytes per query launch from the committed counter summary
    (FETCH_SIZE, WRITE_SIZE scaled by a plain 1 GiB copy), or None when the
    query kernel's sources changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "k_query_c3_counters.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    h = hashlib.sha256()
    for f in ("query.hip", "lg_internal.h"):
        h.update(open(os.path.join(ROOT, "paper_2511_07418_amd", "csrc", f), "rb").read())
    import re
    m = re.search(r"source sha256: ([0-9a-f]{64})", txt)
    t = re.search(r"HBM traffic per launch \(bytes\): ([0-9]+)", txt)
    if not m or not t or m.group(1) != h.hexdigest():
        return None
    return int(t.group(1))


def counter_summary(name: str, sources: tuple) -> dict | None:
    """Per-launch counter values (lines ``- <key> per launch: <number>``) of a
    committed counter summary under profiles/, or None when it is missing or
    the kernel sources changed since it was taken (its ``source sha256`` line
    is the sha256 of ``sources`` in order)."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    h = hashlib.sha256()
    for f in sources:
        h.update(open(os.path.join(ROOT, "paper_2511_07418_amd", "csrc", f), "rb").read())
    m = re.search(r"source sha256: ([0-9a-f]{64})", txt)
    if not m or m.group(1) != h.hexdigest():
        return None
    return {k: float(v) for k, v in re.findall(r"^- ([A-Za-z0-9_ ]+?) per launch: ([0-9.eE+-]+)", txt, re.M)}


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def build_flops(w, vectors: int, dropped: int) -> float:
    """FP32 FLOPs of the field build as the kernel computes them (FMA = 2):
    per (joint sample, link) the joint frame (two 3x4 products, 63 each, the
    first joint of a finger has one; Rodrigues 34) and the composite window
    map (84); per contact vector the window map (18); per contact vector inside
    the window the normal (15) and the nearest of the B bin centres by their
    definition (5 B)."""
    hand, S, B = w.hand, w.field.samples, w.field.bins
    per_sample = 0
    for f in range(hand.n_fingers):
        d = len(hand.finger_joints(f))
        per_sample += d * (63 + 34 + 84) + (d - 1) * 63
    return float(S) * per_sample + 18.0 * vectors + (15.0 + 5.0 * B) * (vectors - dropped)


def realize_flops_per_set(w) -> float:
    """Algorithmic FP32 FLOPs per accepted set (FMA = 2): 10 iterations x sum
    over fingers of (40 d FK + 12 d Jacobian + 6 d^2 J^T J + d^3/3 Cholesky)
    multiply-adds, and the penetration test's axis samples (one per mm, ends
    included) at 63 FLOP each (two rigid transforms, trilinear weights and
    seven interpolations)."""
    hand, it = w.hand, int(w.ik.iters)
    fma = 0.0
    for f in range(hand.n_fingers):
        d = len(hand.finger_joints(f))
        fma += 40 * d + 12 * d + 6 * d * d + d ** 3 / 3.0
    cap = hand.capsule.astype(np.float64)
    L = np.linalg.norm(cap[:, 3:6] - cap[:, 0:3], axis=1)
    samples = float(np.sum(np.ceil(L / 1e-3) + 1))
    return 2.0 * it * fma + 63.0 * samples


def serve_bench(torch, lg, rate: float, seconds: float, seed: int = 0, alone_sample: int = 40,
                n_requests: int = 0, batched: bool = True, slots: int = 0, chunk: int = 4096,
                mix: str = "c4", active: int = 8) -> dict:
    """Serving stream: Poisson arrivals at ``rate`` req/s for ``seconds``
    (or exactly ``n_requests`` arrivals), on a server in batched or
    per-stream mode.

    Each request is a sphere (R = 40 mm) or a superquadric (axes U[30,80] mm,
    exponents U[0.3,2]) with N log-uniform in [2k, 64k] points, a pose budget
    log-uniform in [1k, 64k] and either the 16-DOF or the 22-DOF hand, whose
    fields (64^3 @ 3 mm, 64 bins, S = 262,144, with witnesses) are both
    resident.  D = 32 draws per pose, k = number of fingers, mu = 0.5, 8-edge
    cones; accepted sets run IK + penetration against the object's 64^3 SDF.
    Latency = completion - submission on the server clock.  A sample of the
    same requests is then run one at a time ("alone")."""
    import synth
    rng = np.random.default_rng(seed + 4242)
    hands = {16: synth.hand_c2(seed), 22: synth.hand_c3(seed)}
    fields = {}
    for dof, hnd in hands.items():
        fp = synth.FieldParams(samples=262144, seed=seed, grid=64, h=0.003, bins=64,
                               grid_frame=synth.grid_frames(hnd, 64, 0.003))
        fields[dof] = lg.lg_build_field(hnd, fp, keep_witness=True)
    sph = synth.sphere_object(0.04, 65536)
    pool = [(sph, synth.sdf_sphere(0.04))]
    for i in range(2):
        o = synth.superquadric_object(seed + i, 65536)
        pool.append((o, synth.sdf_superquadric(o)))
    ik = synth.IKParams()
    n_req = n_requests if n_requests > 0 else max(1, int(rng.poisson(rate * seconds)))
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=n_req))
    reqs = []
    for r in range(n_req):
        obj, sdf = pool[0] if rng.uniform() < 0.5 else pool[1 + int(rng.integers(0, len(pool) - 1))]
        n_hi, P_hi = (65536, 65536) if mix == "c4" else (4096, 2048)
        n = int(np.exp(rng.uniform(np.log(2048), np.log(n_hi))))
        P = int(np.exp(rng.uniform(np.log(1024), np.log(P_hi))))
        sel = np.sort(rng.choice(obj.n, size=n, replace=False))  # keeps the Morton order
        dof = 16 if rng.uniform() < 0.5 else 22
        sp = synth.SearchParams(draws=32, k=hands[dof].n_fingers, mu=0.5, m_edges=8, eps=1e-3, seed=seed,
                                moment_scale=obj.rho)
        reqs.append((arrivals[r], (fields[dof], obj.pts[sel], obj.nrm[sel], synth.palm_poses(P, seed + 1000 + r),
                                   sp, 1 + r, ik, sdf)))

    def make(srv, a):
        f, p, nm, po, sp, rid, ik_, sdf_ = a
        return srv.make_request(f, p, nm, po, sp, rid, ik=ik_, sdf=sdf_)

    mode = "batched" if batched else "streams"
    srv = lg.Server(budget_bytes=48 << 30, max_active=active, chunk_poses=chunk, batched=batched,
                    batch_slots=slots)
    built = [make(srv, a) for _, a in reqs]
    print(f"serve {mode} {rate:g} req/s: {n_req} requests over {arrivals[-1]:.1f} s", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    tickets = []
    for i, ((arr, _), (req, keep)) in enumerate(zip(reqs, built)):
        dt = arr - (time.perf_counter() - t0)
        if dt > 0:
            time.sleep(dt)
        tickets.append(srv.submit(req))
        if (i + 1) % 100 == 0:
            print(f"  submitted {i + 1}/{n_req} at {time.perf_counter() - t0:.1f} s, "
                  f"completed {srv.stats()['completed']}", file=sys.stderr, flush=True)
    res = [srv.wait(t, 600.0) for t in tickets]
    assert all(r["state"] == lg.LG_REQ_DONE for r in res), "serving request did not complete"
    lat = np.array([r["t_done"] - r["t_submit"] for r in res]) * 1e3
    span = max(r["t_done"] for r in res) - min(r["t_submit"] for r in res)
    n_valid = sum(r["n_valid"] for r in res)
    st = srv.stats()
    srv.destroy()
    # a sample of the same requests, one at a time
    srv = lg.Server(budget_bytes=48 << 30, max_active=active, chunk_poses=chunk, batched=batched,
                    batch_slots=slots)
    idx = np.linspace(0, n_req - 1, min(alone_sample, n_req)).astype(int)
    alone, alone_valid, same = [], 0, True
    for i in idx:
        req, keep = make(srv, reqs[i][1])
        r = srv.wait(srv.submit(req), 600.0)
        alone.append(r["t_done"] - r["t_submit"])
        alone_valid += r["n_valid"]
        same &= (r["n_acc"], r["n_valid"], r["acc_hash"]) == (res[i]["n_acc"], res[i]["n_valid"],
                                                              res[i]["acc_hash"])
    srv.destroy()
    for f in fields.values():
        f.release()
    alone = np.array(alone)
    return {"mode": mode, "batch_slots": (slots or 4) if batched else None, "max_active": active, "rate_rps": rate, "requests": n_req, "poses": int(sum(len(a[3]) for _, a in reqs)),
            "span_s": span, "batches": int(st["batches"]),
            "chunks_per_batch": (st["batched_chunks"] / st["batches"]) if st["batches"] else None,
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "valid_grasps": int(n_valid), "valid_grasps_per_s": n_valid / span,
            "peak_bytes": int(st["peak_bytes"]),
            "alone_sample": len(idx), "alone_p50_ms": float(np.percentile(alone, 50) * 1e3),
            "alone_p99_ms": float(np.percentile(alone, 99) * 1e3),
            "alone_valid_grasps_per_s": alone_valid / float(alone.sum()),
            "alone_equals_mix": bool(same),
            "chunk_poses": chunk,
            "mix": ("sphere / superquadric 50/50, N log-U[2k,64k], poses log-U[1k,64k], " if mix == "c4" else
                    "sphere / superquadric 50/50, N log-U[2k,4k], poses log-U[1k,2k], ") +
                   "16/22-DOF hands 50/50, D=32, IK + SDF penetration"}


PROP_POINTS = 2048      # proposer input: seeded subsample of the object's points
PROP_POSES = 4096       # pose budget per object, learned and uniform alike
PROP_TARGETS = 64       # training targets kept per object (valid-grasp poses)


def _c2_object(seed: int):
    """A C2 superquadric (N = 16,384) and its 64^3 SDF; runs in a CPU worker."""
    import synth
    o = synth.superquadric_object(seed, 16384)
    return seed, o, synth.sdf_superquadric(o, workers=1)


def _prop_input(torch, obj, seed: int):
    rng = np.random.default_rng(seed + 77)
    sel = np.sort(rng.choice(obj.n, size=PROP_POINTS, replace=False))
    x = np.concatenate([obj.pts[sel], obj.nrm[sel]], axis=1).astype(np.float32)
    return torch.from_numpy(x).cuda()


def _coverage(torch, pipe, ids, obj, cell: float = 0.01) -> tuple:
    """Spread of the valid grasps of one object: (fraction of the object's
    occupied surface cells, edge ``cell``, holding a contact of some valid
    grasp; number of distinct palm-pose cells: the palm origin in the object
    frame on the same grid, times the palm's approach axis (+z) in one of 96
    cube-map directions, 6 faces x 4 x 4)."""
    p = torch.from_numpy(obj.pts).cuda()
    c = torch.floor(p / cell).long() + (1 << 10)
    key = (c[:, 0] << 22) | (c[:, 1] << 11) | c[:, 2]
    occ, pt_cell = torch.unique(key, return_inverse=True)
    if ids.numel() == 0:
        return 0.0, 0
    k = pipe.sbuf.set_pt.shape[-1]
    sets = pipe.sbuf.set_pt.view(-1, k)[ids.long()].reshape(-1).long()
    surf = torch.unique(pt_cell[sets[sets >= 0]]).numel() / occ.numel()
    P = pipe.poses[(ids.long() // int(pipe.sp.draws))].view(-1, 3, 4).double()
    R, t = P[:, :, :3], P[:, :, 3]
    o = -(R.transpose(1, 2) @ t.unsqueeze(-1)).squeeze(-1)   # palm origin, object frame
    z = R[:, 2, :]                                            # palm +z axis, object frame
    a = z.abs().argmax(dim=1)
    major = z.gather(1, a[:, None]).squeeze(1)
    face = 2 * a + (major < 0).long()
    uv = torch.stack([z[:, 1], z[:, 2], z[:, 0], z[:, 2], z[:, 0], z[:, 1]], 1).view(-1, 3, 2)
    uv = uv[torch.arange(len(a), device=z.device), a] / major.abs()[:, None]
    b = torch.clamp(((uv + 1.0) * 2.0).long(), 0, 3)
    dirbin = face * 16 + b[:, 0] * 4 + b[:, 1]
    oc = torch.floor(o / cell).long() + (1 << 10)
    pk = (((oc[:, 0] << 22) | (oc[:, 1] << 11) | oc[:, 2]) * 96) + dirbin
    return float(surf), int(torch.unique(pk).numel())


def _diversity(torch, pipe, ids) -> int:
    """Distinct sorted point-index k-tuples among the valid grasps."""
    if ids.numel() == 0:
        return 0
    sets = pipe.sbuf.set_pt.view(-1, pipe.sbuf.set_pt.shape[-1])[ids.long()]
    return int(torch.unique(torch.sort(sets, dim=1).values, dim=0).shape[0])


def encoder_bench(torch, lg, X, seed: int = 0, reps: int = 10) -> dict:
    """Forward pass of 512 objects x 2048 points (the rows of X repeated):
    the encoder's dense BF16 MFMA work, then the pooled head.  The FLOP count
    is the encoder's alone (the head adds 0.25 %)."""
    big = lg.Proposer(max_batch=512, max_points=PROP_POINTS, max_targets=1, seed=seed)
    xb = X[torch.arange(512, device="cuda") % X.shape[0]].contiguous()
    for _ in range(3):
        big.forward(xb)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for _ in range(reps):
        big.forward(xb)
    ev[1].record()
    torch.cuda.synchronize()
    f_ms = ev[0].elapsed_time(ev[1]) / reps
    flops = 2.0 * 512 * PROP_POINTS * (6 * 128 + 128 * 256)
    big.release()
    return {"objects": 512, "points": PROP_POINTS, "forward_ms": f_ms, "encoder_gflop": flops / 1e9,
            "tflops": flops / (f_ms * 1e-3) / 1e12, "peak_tflops": 2500.0,
            "frac": flops / (f_ms * 1e-3) / 1e12 / 2500.0}


def proposer_bench(torch, lg, pool, n_train: int, n_eval: int, epochs: int, seed: int = 0) -> dict:
    """C5: train the proposer on the valid grasps of uniform search over
    n_train C2 objects, then compare learned and uniform proposals on n_eval
    held-out objects at an equal pose budget under the unchanged checks."""
    import synth
    from paper_2511_07418_amd.pipeline import Pipeline
    hand = synth.hand_c2(seed)
    fp = synth.FieldParams(samples=262144, seed=seed, grid=64, h=0.003, bins=64,
                           grid_frame=synth.grid_frames(hand, 64, 0.003))
    field = lg.lg_build_field(hand, fp, keep_witness=True)
    ik = synth.IKParams()

    def run(obj, sdf, poses):
        sp = synth.SearchParams(draws=32, k=hand.n_fingers, mu=0.5, m_edges=8, eps=1e-3, seed=seed,
                                moment_scale=obj.rho)
        pipe = Pipeline(field, obj.pts, obj.nrm, poses, sp, ik=ik, sdf=sdf)
        return pipe

    # ---- training data: valid grasps of uniform search ----------------------------
    t0 = time.perf_counter()
    xs, ys = [], []
    n_valid_train = 0
    for i, (s_, obj, sdf) in enumerate(pool.imap(_c2_object, range(n_train), chunksize=4)):
        pipe = run(obj, sdf, synth.palm_poses(PROP_POSES, s_ + 1))
        pipe.step()
        ids = pipe.valid_sets()
        n_valid_train += int(ids.numel())
        if ids.numel():
            g = (ids // 32).long()
            rng = np.random.default_rng(s_ + 5)
            pick = torch.from_numpy(rng.choice(int(g.numel()), size=min(PROP_TARGETS, int(g.numel())),
                                               replace=False)).cuda()
            P = pipe.poses[g[pick]]
            y = torch.cat([P[:, [0, 4, 8]], P[:, [1, 5, 9]], P[:, [3, 7, 11]] / 0.1], dim=1)
            xs.append(_prop_input(torch, obj, s_))
            ys.append(y)
        if (i + 1) % 100 == 0:
            print(f"[proposer] data {i + 1}/{n_train} objects, {len(xs)} with valid grasps, "
                  f"{time.perf_counter() - t0:.0f}s", file=sys.stderr, flush=True)
    t_data = time.perf_counter() - t0
    # ---- training -------------------------------------------------------------------
    Bt = 32
    prop = lg.Proposer(max_batch=Bt, max_points=PROP_POINTS, max_targets=Bt * PROP_TARGETS, seed=seed)
    X = torch.stack(xs)
    rng = np.random.default_rng(seed + 99)
    losses = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for ep in range(epochs):
        order = rng.permutation(len(xs))
        ep_loss = []
        for j in range(0, len(order) - Bt + 1, Bt):
            idx = order[j:j + Bt]
            tg = torch.cat([ys[k] for k in idx]).contiguous()
            off = torch.from_numpy(np.concatenate([[0], np.cumsum([len(ys[k]) for k in idx])]).astype(np.int32)).cuda()
            ep_loss.append(prop.train_step(X[torch.from_numpy(idx).cuda()].contiguous(), tg, off, 1e-3))
        losses.append(float(torch.stack(ep_loss).mean().cpu()))
        print(f"[proposer] epoch {ep + 1}/{epochs} loss {losses[-1]:.3f}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    # ---- evaluation on held-out objects ---------------------------------------------------
    res = {kind: {"valid": 0, "diversity": 0, "surface": 0.0, "pose_cells": 0, "s": 0.0, "per_obj": []}
           for kind in ("uniform", "learned")}
    ev = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    held = []
    for i, (s_, obj, sdf) in enumerate(pool.imap(_c2_object, range(100000, 100000 + n_eval), chunksize=2)):
        x = _prop_input(torch, obj, s_)
        held.append((s_, obj, sdf, x))
        for kind in ("uniform", "learned"):
            if kind == "uniform":
                poses = torch.from_numpy(synth.palm_poses(PROP_POSES, s_ + 1)).cuda()
            else:
                poses = torch.empty((PROP_POSES, 12), dtype=torch.float32, device="cuda")
            pipe = run(obj, sdf, poses)
            torch.cuda.synchronize()
            ev[0].record()
            if kind == "learned":
                prop.sample(x, PROP_POSES, seed=s_, uniform_frac=0.1, out=pipe.poses)
            pipe.step()
            ev[1].record()
            torch.cuda.synchronize()
            ids = pipe.valid_sets()
            r = res[kind]
            r["valid"] += int(ids.numel())
            r["diversity"] += _diversity(torch, pipe, ids)
            surf, cells = _coverage(torch, pipe, ids, obj)
            r["surface"] += surf
            r["pose_cells"] += cells
            r["s"] += ev[0].elapsed_time(ev[1]) * 1e-3
            r["per_obj"].append(int(ids.numel()))
    out = {"train_objects": n_train, "train_objects_with_valid": len(xs), "train_valid_grasps": n_valid_train,
           "targets": int(sum(len(y) for y in ys)), "epochs": epochs, "loss_first_epoch": losses[0],
           "loss_last_epoch": losses[-1], "data_s": t_data, "train_s": t_train, "eval_objects": n_eval,
           "pose_budget": PROP_POSES, "uniform_frac": 0.1}
    for kind, r in res.items():
        out[kind] = {"valid_grasps": r["valid"], "valid_per_object": r["valid"] / n_eval,
                     "valid_grasps_per_s": r["valid"] / r["s"], "distinct_contact_sets": r["diversity"],
                     "contact_surface_coverage": r["surface"] / n_eval,
                     "palm_pose_cells_per_object": r["pose_cells"] / n_eval,
                     "seconds": r["s"]}
    pu, pl = np.array(res["uniform"]["per_obj"]), np.array(res["learned"]["per_obj"])
    out["objects_learned_ge_uniform"] = int((pl >= pu).sum())
    # the same held-out objects as a back-to-back request stream through the
    # serving loop; pose generation (CPU for uniform, proposer forward +
    # sampling on the GPU for learned) is inside the timed span
    out["serving"] = {}
    for kind in ("uniform", "learned"):
        srv = lg.Server(budget_bytes=32 << 30, max_active=8, chunk_poses=PROP_POSES)
        keep, tickets = [], []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for r_, (s_, obj, sdf, x) in enumerate(held):
            if kind == "uniform":
                poses = synth.palm_poses(PROP_POSES, s_ + 1)
            else:
                poses = prop.sample(x, PROP_POSES, seed=s_, uniform_frac=0.1).cpu().numpy()
            sp = synth.SearchParams(draws=32, k=hand.n_fingers, mu=0.5, m_edges=8, eps=1e-3, seed=seed,
                                    moment_scale=obj.rho)
            req, kp = srv.make_request(field, obj.pts, obj.nrm, poses, sp, 1 + r_, ik=ik, sdf=sdf)
            keep.append((req, kp))
            tickets.append(srv.submit(req))
        res = [srv.wait(t, 600.0) for t in tickets]
        wall = time.perf_counter() - t0
        srv.destroy()
        assert all(r["state"] == lg.LG_REQ_DONE for r in res)
        lat = np.array([r["t_done"] - r["t_submit"] for r in res]) * 1e3
        nv = int(sum(r["n_valid"] for r in res))
        out["serving"][kind] = {"valid_grasps": nv, "seconds": wall, "valid_grasps_per_s": nv / wall,
                                "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99))}
    out["serving"]["valid_per_s_ratio"] = (out["serving"]["learned"]["valid_grasps_per_s"] /
                                           out["serving"]["uniform"]["valid_grasps_per_s"])
    out["encoder_forward"] = encoder_bench(torch, lg, X, seed)
    out["valid_per_s_ratio"] = out["learned"]["valid_grasps_per_s"] / max(out["uniform"]["valid_grasps_per_s"], 1e-9)
    prop.release()
    field.release()
    return out


def cpu_baseline(w, n_all: int, n_one: int) -> dict:
    """The FP64 oracle, as it stands, on the same workload: its own field built
    with the GPU's joint-sample count S (untimed), then query, draws, verdicts,
    compaction and (with an SDF) IK + penetration on the first ``n_all``
    poses with every host thread, and on the first ``n_one`` poses with one."""
    import oracle

    fld = oracle.build_field(w.hand, w.field, witness=w.ik is not None, flags=False)
    all_threads = oracle.get_threads()

    def run(n: int) -> tuple:
        poses = w.poses[:n]
        t0 = time.perf_counter()
        Q = oracle.query(w.hand, w.field, fld["bits"], w.obj.pts, w.obj.nrm, poses, flags=False)
        spt, sln = oracle.draw(w.hand, w.field, fld["bits"], w.obj.pts, w.obj.nrm, poses, Q["dom_bits"],
                               Q["dom_count"], w.search)
        V = oracle.verdicts(w.obj.pts, w.obj.nrm, spt, w.search)
        acc = oracle.compact(V["verdict"])
        n_valid = len(acc)
        if w.ik is not None and len(acc):
            k = w.search.k
            R = oracle.realize(w.hand, w.field, fld["wit"], w.sdf, w.obj.pts, w.obj.nrm, poses,
                               spt.reshape(-1, k), sln.reshape(-1, k), w.search, acc, w.ik)
            n_valid = int(R["valid"].sum())
        return n_valid, time.perf_counter() - t0

    v_all, t_all = run(n_all)
    oracle.set_threads(1)
    try:
        v_one, t_one = run(n_one)
    finally:
        oracle.set_threads(all_threads)
    return {"value": v_all / t_all, "unit": "valid grasps/s", "cores": all_threads, "kind": "oracle",
            "sample": f"first {n_all} of {w.poses.shape[0]} poses of the same workload (full N and D, the "
                      f"oracle's own field at S = {w.field.samples}, built untimed): {v_all} valid grasps in "
                      f"{t_all:.2f} s on {all_threads} threads",
            "cpu_model": cpu_model(), "seconds": t_all, "poses_per_s": n_all / t_all,
            "single_thread": {"value": v_one / t_one, "unit": "valid grasps/s", "cores": 1,
                              "sample": f"first {n_one} poses: {v_one} valid grasps in {t_one:.2f} s",
                              "seconds": t_one, "poses_per_s": n_one / t_one}}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    pool = None
    if args.mode == "proposer":
        # CPU workers for the object and SDF generators, forked before the GPU is touched
        import multiprocessing as mp
        pool = mp.get_context("fork").Pool(min(16, os.cpu_count() or 1))
    import torch

    import synth
    from paper_2511_07418_amd import lg
    from paper_2511_07418_amd.pipeline import Pipeline

    torch.cuda.set_device(0)
    if args.mode == "proposer":
        out = proposer_bench(torch, lg, pool, args.train_objects, args.eval_objects, args.epochs, args.seed)
        pool.close()
        print(json.dumps({"proposer": out}))
        return
    if args.mode == "encoder":
        # proposer forward alone: random-init weights, 8 c2 objects' point subsamples repeated
        objs = [synth.superquadric_object(args.seed + i, 16384) for i in range(8)]
        X = torch.stack([_prop_input(torch, o, args.seed + i) for i, o in enumerate(objs)])
        print(json.dumps({"encoder_forward": encoder_bench(torch, lg, X, args.seed, reps=max(args.steps, 1))}))
        return
    if args.mode == "serve":
        for rate in [float(r) for r in args.serve_rates.split(",")]:
            for mode in args.serve_modes.split(","):
                if mode not in ("batched", "streams"):
                    raise SystemExit(f"unknown serve mode {mode!r}")
                r = serve_bench(torch, lg, rate, args.serve_seconds, args.seed, args.serve_alone,
                                args.serve_requests, batched=(mode == "batched"), slots=args.serve_slots,
                                chunk=args.serve_chunk, mix=args.serve_mix, active=args.serve_active)
                print(json.dumps({"serving": r}), flush=True)
        return
    w = synth.workload(args.workload, seed=args.seed, with_sdf=(args.workload == "c3"))
    if args.self_collision and w.ik is not None:
        import dataclasses
        w.ik = dataclasses.replace(w.ik, self_collision=1)
    if args.opt_outer > 0:
        import dataclasses
        w.search = dataclasses.replace(w.search, opt_outer=args.opt_outer, opt_inner=args.opt_inner,
                                       opt_sigma=args.opt_sigma)
    if args.k > 0:
        import dataclasses
        w.search = dataclasses.replace(w.search, k=args.k)
    palm = synth.palm_for(args.workload) if args.palm_prob > 0 else None
    if palm is not None and w.sdf is None:
        raise SystemExit("--palm-prob needs the object's SDF (workload c3)")
    t_build = time.perf_counter()
    field = lg.lg_build_field(w.hand, w.field, keep_witness=w.ik is not None, palm=palm)
    t_build = time.perf_counter() - t_build
    cos_hit = math.cos(math.radians(args.cone_deg)) if args.cone_deg > 0 else None
    obj_pts, obj_nrm, concave = w.obj.pts, w.obj.nrm, None
    sdf_vals = sdf_s = None
    if w.sdf is not None:
        sdf_vals = torch.from_numpy(np.ascontiguousarray(w.sdf.values, np.float32)).cuda()
        sdf_s = lg.sdf_struct(w.sdf, sdf_vals)
    p_soa = torch.from_numpy(np.ascontiguousarray(w.obj.pts.T)).cuda()
    n_soa = torch.from_numpy(np.ascontiguousarray(w.obj.nrm.T)).cuda()
    if args.concave_filter:
        if w.sdf is None:
            raise SystemExit("--concave-filter needs the object's SDF (workload c3)")
        lg.lg_concave_filter(sdf_s, p_soa, n_soa)          # warm-up (module load)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        cr = lg.lg_concave_filter(sdf_s, p_soa, n_soa, 0.008, 4, 0.001)
        e1.record()
        torch.cuda.synchronize()
        nk = int(cr.n_kept.item())
        p_soa, n_soa = lg.lg_gather_points(p_soa, n_soa, cr.kept_idx, nk)
        obj_pts, obj_nrm = p_soa.t().cpu().numpy(), n_soa.t().cpu().numpy()
        concave = {"box_edge_m": 0.008, "lattice": 4, "max_depth_m": 0.001, "kept": nk, "of": int(w.obj.n),
                   "filter_ms": e0.elapsed_time(e1)}
        print(f"[bench] concave filter kept {nk} of {w.obj.n} points in {concave['filter_ms']:.3f} ms",
              file=sys.stderr, flush=True)
    # placement (Sec. 5.1): the poses are the step's input, made before the timed region
    poses = w.poses
    if args.placement == "exhaustive":
        poses = lg.lg_place_exhaustive(field, p_soa, n_soa, len(w.poses), seed=args.seed + 1)
        torch.cuda.synchronize()
    palm_pt, palm_info = None, None
    if palm is not None:
        if not isinstance(poses, torch.Tensor):
            poses = torch.from_numpy(np.ascontiguousarray(poses, np.float32)).cuda()
        palm_pt = lg.lg_place_palm(field, sdf_s, p_soa, n_soa, poses, args.palm_prob, 0.002, seed=args.seed + 2)
        torch.cuda.synchronize()
        pc = palm_pt.cpu().numpy()
        palm_info = {"prob": args.palm_prob, "placed": int((pc >= 0).sum()), "rejected": int((pc == -2).sum()),
                     "radius_m": palm.radius, "margin_m": 0.002}
        print(f"[bench] palm placements: {palm_info['placed']} kept, {palm_info['rejected']} rejected",
              file=sys.stderr, flush=True)
    if args.extend > 0 and (w.ik is None or int(w.search.k) + args.extend > w.hand.n_fingers):
        raise SystemExit("--extend needs the c3 workload and --k + --extend <= the number of fingers")
    pipe = Pipeline(field, obj_pts, obj_nrm, poses, w.search, ik=w.ik, sdf=w.sdf, cos_hit=cos_hit, palm_pt=palm_pt,
                    extend_k=args.extend)
    print(f"[bench] {args.workload}: field built in {t_build:.2f}s ({field.info()['bits_set']} bits), "
          f"P={pipe.P} N={pipe.N}", file=sys.stderr, flush=True)

    if args.mode == "search":
        pipe.query()
        for _ in range(args.steps):
            pipe.search()
        torch.cuda.synchronize()
        print(f"[bench] search-only run done: {args.steps} launches", file=sys.stderr, flush=True)
        return
    if args.mode == "query":
        # counter runs: the query kernel alone, then a plain copy of known size
        # (1 GiB read + 1 GiB written) whose FETCH_SIZE / WRITE_SIZE calibrate
        # the counters' units
        for _ in range(args.steps):
            pipe.query()
        src = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"[bench] query-only run done: {args.steps} launches", file=sys.stderr, flush=True)
        return

    if args.mode == "multipass":
        # Sec. 5.7 multi-pass generation: one query, then R resamplings of the
        # cached domains (request ids 1..R), each with the verdicts and realize.
        # Timed: the kernels only; the valid counts are summed on the device.
        pipe.step()
        R = args.passes
        rows = torch.arange(pipe.max_acc, device="cuda", dtype=torch.int32)
        counts = torch.zeros(R, dtype=torch.int64, device="cuda")
        # one untimed pass with the device-side count (loads every kernel it uses)
        pipe.search(request_id=R + 1)
        pipe.realize()
        counts[0] = ((pipe.rbuf.valid != 0) & (rows < pipe.sbuf.n_acc)).sum()
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record()
        pipe.query()
        for r in range(R):
            pipe.search(request_id=r + 1)
            pipe.realize()
            counts[r] = ((pipe.rbuf.valid != 0) & (rows < pipe.sbuf.n_acc)).sum()
        ev[1].record()
        torch.cuda.synchronize()
        ms = ev[0].elapsed_time(ev[1])
        n_valid = int(counts.sum().item())
        # distinct valid grasps over the passes (recomputed, untimed)
        keys = []
        for r in range(R):
            pipe.search(request_id=r + 1)
            pipe.realize()
            ids = pipe.valid_sets()
            sets = pipe.sbuf.set_pt.view(-1, pipe.sbuf.set_pt.shape[-1])[ids.long()]
            g = (ids // pipe.sbuf.set_pt.shape[1]).long()[:, None]
            keys.append(torch.cat([g, torch.sort(sets.long(), dim=1).values], dim=1))
        distinct = int(torch.unique(torch.cat(keys), dim=0).shape[0])
        print(json.dumps({"multipass": {"workload": args.workload, "passes": R, "ms": ms,
                                        "valid_grasps": n_valid, "distinct_valid_grasps": distinct,
                                        "valid_grasps_per_s": n_valid / (ms * 1e-3),
                                        "note": "one query, then R draws + verdicts + realize on the cached "
                                                "domains (request ids 1..R)"}}))
        return

    for _ in range(args.warmup):
        pipe.step()
    torch.cuda.synchronize()

    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(args.steps)]
    valid = []
    t0 = time.perf_counter()
    for s in range(args.steps):
        e = ev[s]
        e[0].record()
        pipe.query()
        e[1].record()
        pipe.search()
        e[2].record()
        pipe.realize()
        e[3].record()
        if pipe.extend_k > 0:
            pipe.extend()
        e[4].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    n_valid = pipe.valid_count()
    n_acc = pipe.n_acc()
    st = np.array([[e[i].elapsed_time(e[i + 1]) for i in range(4)] for e in ev])  # ms
    ms_per_step = wall * 1000.0 / args.steps
    value = n_valid / (ms_per_step / 1000.0)

    # Query roofline (HBM, the gather bound of the method).  Algorithmic bytes
    # per launch: 4 B per in-window (pose, point, finger) lookup -- the word of
    # the finger's merged table (the OR of its links' tables, Sec. 5.3) that
    # holds the query's bin -- plus the domain bits written (P*F*ceil(N/32)*4),
    # the counts (4*P*F), 48 B per pose and 24 B per point.  The per-link
    # figure (B/8 bytes per in-window (pose, point, link) lookup, as if each
    # link's table were read) is kept as a labelled diagnostic.
    W = w.field.bins // 8
    per_finger = in_window_lookups(torch, pipe, w)
    dof = w.hand.dof
    link_lookups = sum(c * d for c, d in zip(per_finger, dof))
    finger_lookups = sum(per_finger)
    F = w.hand.n_fingers
    NW = (pipe.N + 31) // 32
    out_bytes = pipe.P * F * NW * 4 + pipe.P * F * 4 + pipe.P * 48 + pipe.N * 24
    alg_bytes = finger_lookups * 4 + out_bytes
    link_bytes = link_lookups * W + out_bytes
    q_ms = float(st[:, 0].mean())
    q_s = q_ms * 1e-3
    achieved = alg_bytes / q_s / 1e9
    # counters of the default c3 launch (canonical poses, all points, nearest bin)
    canonical = (args.placement == "canonical" and not args.cone_deg and not args.concave_filter
                 and args.workload == "c3" and args.seed == 0 and not args.palm_prob)
    qc = counter_summary("k_query_c3_counters.md", ("query.hip", "lg_internal.h")) if canonical else None
    issue = None
    if qc:
        miss_bytes = qc["TCC_MISS_sum"] * 128.0
        issue = {"valu_wave_instr_per_launch": qc["SQ_INSTS_VALU"], "salu_instr_per_launch": qc["SQ_INSTS_SALU"],
                 "valu_g_per_s": qc["SQ_INSTS_VALU"] / q_s / 1e9,
                 "valu_issue_limit_g_per_s": 1024 * 2.4 / 4.0,
                 "l2_miss_bytes_per_launch": miss_bytes, "l2_miss_gbps": miss_bytes / q_s / 1e9,
                 "l2_miss_frac_of_hbm_peak": miss_bytes / q_s / 1e9 / HBM_PEAK_GBPS,
                 "l2_hit_rate": qc["TCC_HIT_sum"] / (qc["TCC_HIT_sum"] + qc["TCC_MISS_sum"])}
    # FP32 FLOP fractions of FK (the field build) and IK (realize) against the
    # 157.3 TFLOP/s FP32 vector peak: algorithmic counts (build_flops,
    # realize_flops_per_set) and the VALU FP32 counters (64 lanes per
    # wave-instruction, FMA = 2) of the committed summary
    finfo = field.info()
    fc = counter_summary("fp32_flops_c3.md", ("field.hip", "realize.hip", "lg_internal.h")) if canonical else None
    r_ms = float(st[:, 2].mean())
    fp32 = {"peak_tflops": FP32_PEAK_TFLOPS}
    b_ms = float(finfo["build_kernel_ms"])
    if b_ms > 0:
        bf = build_flops(w, int(finfo["vectors"]), int(finfo["dropped"]))
        fp32["fk_field_build"] = {"kernel": "k_field_build", "ms": b_ms, "alg_gflop": bf / 1e9,
                                  "alg_tflops": bf / (b_ms * 1e-3) / 1e12,
                                  "alg_frac": bf / (b_ms * 1e-3) / 1e12 / FP32_PEAK_TFLOPS}
        if fc:
            cf = fc["k_field_build SQ_INSTS_VALU_FLOPS_FP32"] * 64.0
            fp32["fk_field_build"].update({"counter_gflop": cf / 1e9,
                                           "counter_frac": cf / (b_ms * 1e-3) / 1e12 / FP32_PEAK_TFLOPS})
    if w.ik is not None and n_acc > 0:
        rf = realize_flops_per_set(w) * n_acc
        fp32["ik_realize"] = {"kernel": "k_realize", "ms": r_ms, "sets": n_acc, "alg_gflop": rf / 1e9,
                              "alg_tflops": rf / (r_ms * 1e-3) / 1e12,
                              "alg_frac": rf / (r_ms * 1e-3) / 1e12 / FP32_PEAK_TFLOPS}
        if fc:
            cf = fc["k_realize SQ_INSTS_VALU_FLOPS_FP32"] * 64.0
            fp32["ik_realize"].update({"counter_gflop": cf / 1e9,
                                       "counter_frac": cf / (r_ms * 1e-3) / 1e12 / FP32_PEAK_TFLOPS})
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "valid grasps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {DESCR[args.workload]}", "poses_per_step": pipe.P,
                   "points": pipe.N, "draws": int(w.search.draws), "seed": args.seed,
                   "contact_opt": ({"rounds": args.opt_outer, "candidates": args.opt_inner,
                                    "sigma_m": args.opt_sigma} if args.opt_outer > 0 else None),
                   "self_collision": bool(args.self_collision), "placement": args.placement,
                   "cone_deg": args.cone_deg or None, "contacts": int(w.search.k), "concave_filter": concave,
                   "second_round_contacts": args.extend or None,
                   "palm": palm_info},
        "valid_per_step": n_valid,
        "accepted_sets_per_step": n_acc,
        "stage_ms": {"query": q_ms, "search": float(st[:, 1].mean()), "realize": float(st[:, 2].mean()),
                     **({"second_round": float(st[:, 3].mean())} if pipe.extend_k > 0 else {})},
        "query_gbps": achieved,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBPS,
                     "traffic": query_traffic() if canonical else None,
                     "kernel": "k_query", "alg_bytes_per_launch": alg_bytes,
                     "alg_per_unit": "4 B per in-window (pose, point, finger) lookup of the merged finger table, "
                                     "P*F*ceil(N/32)*4 B domain bits, 4*P*F B counts, 48 B per pose, 24 B per point",
                     "in_window_finger_lookups": finger_lookups,
                     "issue": issue,
                     "per_link_diagnostic": {"bytes_per_launch": link_bytes, "gbps": link_bytes / q_s / 1e9,
                                             "in_window_link_lookups": link_lookups,
                                             "note": "B/8 bytes per in-window (pose, point, link) lookup, as if "
                                                     "every link's own table were read; not a roofline"}},
        "fp32_flops": fp32,
    }
    out["poses_per_s"] = pipe.P / (ms_per_step / 1000.0)
    if not args.no_serve:
        pipe = None
        field.release()
        torch.cuda.empty_cache()
        out["serving"] = serve_bench(torch, lg, args.serve_rate, args.serve_seconds, args.seed)
        out["p50_ms"] = out["serving"]["p50_ms"]
        out["p99_ms"] = out["serving"]["p99_ms"]
    if not args.no_cpu_baseline:
        n = args.cpu_poses or {"c1": 256, "c2": 2048, "c3": 5120}[args.workload]
        out["cpu_baseline"] = cpu_baseline(w, n, max(1, n // 16))
    print(json.dumps(out))


if __name__ == "__main__":
    main()
