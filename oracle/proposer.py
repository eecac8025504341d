"""FP64 oracle of the learned palm-pose proposer -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s ``cpu_baseline``
leg may import this module; the HIP library never does and shares no code
with it.

The paper does not specify a proposer: Sec. 5.7 ("Data-driven Search") names
learning where to search as a way to skip unproductive regions and leaves it
unimplemented.  The model below is the stated configuration of this project,
written from the standard definitions it is made of:

* a PointNet-style encoder (Qi et al., CVPR 2017): a shared per-point MLP
  6 -> 128 -> 256 with ReLU, then a max-pool over the points;
* a head 256 -> 256 -> 256 (ReLU) -> 152 emitting an 8-component diagonal
  Gaussian mixture (a mixture density network, Bishop 1994) over the
  9-vector y = (first two columns of R, t / S_T) of a palm pose;
* the 6-D rotation representation and its Gram-Schmidt map back to SO(3)
  (Zhou et al., CVPR 2019);
* sampling with Philox4x32-10 words: the component by inversion of the
  cumulative softmax, the Gaussian by Box-Muller (1958), the uniform fallback
  pose by Shoemake's uniform quaternion (Graphics Gems III, 1992).

Everything is float64 and written for clarity, not speed.  ``bf16=True``
rounds every matrix-product operand to bfloat16 (round to nearest even),
which is the precision in which the GPU takes the max-pool's argmax decision.
"""
from __future__ import annotations

import math

import numpy as np

S_P = 0.1            # m, scale of input point coordinates
S_T = 0.1            # m, scale of the translation part of y
D_IN, H1, H2, HH = 6, 128, 256, 256
M, Y = 8, 9
OUT = M * (1 + 2 * Y)          # 152 = 8 logits + 8x9 means + 8x9 log-sigmas
LS_MIN, LS_MAX = -5.0, 2.0     # clamp of log sigma
PHILOX_TAG = 7                 # third counter word of the proposer's draws

# flat parameter layout (row-major [in][out] weights, then the bias)
LAYERS = [("W1", (D_IN, H1)), ("b1", (H1,)), ("W2", (H1, H2)), ("b2", (H2,)),
          ("Wa", (H2, HH)), ("ba", (HH,)), ("Wb", (HH, HH)), ("bb", (HH,)),
          ("Wc", (HH, OUT)), ("bc", (OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in LAYERS)


def unflatten(flat: np.ndarray) -> dict:
    out, o = {}, 0
    for name, shp in LAYERS:
        n = int(np.prod(shp))
        out[name] = np.asarray(flat[o:o + n], np.float64).reshape(shp)
        o += n
    return out


def flatten(p: dict) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], np.float64).ravel() for name, _ in LAYERS])


def bf16_round(a) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(a, np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def _mm(a, b, bf16: bool):
    if bf16:
        return bf16_round(a) @ bf16_round(b)
    return a @ b


def inputs(pts, nrm) -> np.ndarray:
    """Per-point input row (p / S_P, n)."""
    return np.concatenate([np.asarray(pts, np.float64) / S_P, np.asarray(nrm, np.float64)], axis=1)


# ---------------------------------------------------------------------------
# forward
# ---------------------------------------------------------------------------
def encode(p: dict, x: np.ndarray, bf16: bool = False) -> dict:
    """Shared MLP + max-pool of one object's [N][6] inputs.  The argmax takes
    the lowest point index among equal maxima."""
    z1 = _mm(x, p["W1"], bf16) + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = _mm(h1, p["W2"], bf16) + p["b2"]
    h2 = np.maximum(z2, 0.0)
    arg = np.argmax(h2, axis=0)             # first maximum
    feat = h2[arg, np.arange(h2.shape[1])]
    # gap between the best and the second-best point of each channel,
    # relative to the channel's magnitude (near-ties flag the argmax)
    if h2.shape[0] > 1:
        part = np.partition(h2, h2.shape[0] - 2, axis=0)
        gap = (part[-1] - part[-2]) / np.maximum(np.abs(part[-1]), 1e-30)
    else:
        gap = np.full(h2.shape[1], np.inf)
    return {"z1": z1, "h1": h1, "z2": z2, "feat": feat, "arg": arg, "gap": gap}


def head(p: dict, feat: np.ndarray, bf16: bool = False) -> dict:
    """feat [B][256] -> mixture parameters [B][152]."""
    ua = np.maximum(_mm(feat, p["Wa"], bf16) + p["ba"], 0.0)
    ub = np.maximum(_mm(ua, p["Wb"], bf16) + p["bb"], 0.0)
    o = _mm(ub, p["Wc"], bf16) + p["bc"]
    return {"ua": ua, "ub": ub, "out": o}


def forward(p: dict, xs: list, bf16: bool = False) -> dict:
    enc = [encode(p, x, bf16) for x in xs]
    feat = np.stack([e["feat"] for e in enc])
    hd = head(p, feat, bf16)
    return {"enc": enc, "feat": feat, **hd}


def mixture(o: np.ndarray):
    """(log pi [M], mu [M][Y], log sigma [M][Y] clamped, clamp mask) of one output row."""
    logits = o[:M]
    lp = logits - (logits.max() + np.log(np.exp(logits - logits.max()).sum()))
    mu = o[M:M + M * Y].reshape(M, Y)
    raw = o[M + M * Y:].reshape(M, Y)
    ls = np.clip(raw, LS_MIN, LS_MAX)
    inside = (raw > LS_MIN) & (raw < LS_MAX)
    return lp, mu, ls, inside


def nll(o: np.ndarray, y: np.ndarray) -> float:
    """-log p(y) under the mixture of one output row."""
    lp, mu, ls, _ = mixture(o)
    z = (y[None, :] - mu) / np.exp(ls)
    comp = lp + np.sum(-0.5 * z * z - ls - 0.5 * math.log(2.0 * math.pi), axis=1)
    mx = comp.max()
    return float(-(mx + math.log(np.exp(comp - mx).sum())))


def loss(p: dict, xs: list, targets: np.ndarray, offsets: np.ndarray, bf16: bool = False) -> float:
    """Mean NLL over all targets; object b owns targets offsets[b]:offsets[b+1]."""
    f = forward(p, xs, bf16)
    T = int(offsets[-1])
    tot = 0.0
    for b in range(len(xs)):
        for t in range(int(offsets[b]), int(offsets[b + 1])):
            tot += nll(f["out"][b], targets[t])
    return tot / T


# ---------------------------------------------------------------------------
# backward (the chain rule written out per layer)
# ---------------------------------------------------------------------------
def grad_out(o: np.ndarray, ys: np.ndarray, scale: float) -> np.ndarray:
    """d(scale * sum_t nll(o, y_t)) / d o for one object's output row."""
    lp, mu, ls, inside = mixture(o)
    sig = np.exp(ls)
    g = np.zeros(OUT)
    for y in ys:
        z = (y[None, :] - mu) / sig
        comp = lp + np.sum(-0.5 * z * z - ls - 0.5 * math.log(2.0 * math.pi), axis=1)
        r = np.exp(comp - comp.max())
        r /= r.sum()                                   # responsibilities
        g[:M] += np.exp(lp) - r
        g[M:M + M * Y] += (-r[:, None] * z / sig).ravel()
        g[M + M * Y:] += (r[:, None] * (1.0 - z * z) * inside).ravel()
    return g * scale


def backward(p: dict, xs: list, targets: np.ndarray, offsets: np.ndarray, bf16: bool = False,
             arg_override: dict | None = None) -> tuple[float, dict]:
    """(mean NLL, gradients of every parameter).  ``arg_override`` maps
    (object, channel) -> point index to take another of several equal
    maxima (used where the argmax is a near-tie)."""
    f = forward(p, xs, bf16)
    B, T = len(xs), int(offsets[-1])
    L = 0.0
    dO = np.zeros((B, OUT))
    for b in range(B):
        ys = targets[int(offsets[b]):int(offsets[b + 1])]
        for y in ys:
            L += nll(f["out"][b], y)
        dO[b] = grad_out(f["out"][b], ys, 1.0 / T)
    g = {}
    # head
    g["Wc"] = f["ub"].T @ dO
    g["bc"] = dO.sum(0)
    dub = (dO @ p["Wc"].T) * (f["ub"] > 0)
    g["Wb"] = f["ua"].T @ dub
    g["bb"] = dub.sum(0)
    dua = (dub @ p["Wb"].T) * (f["ua"] > 0)
    g["Wa"] = f["feat"].T @ dua
    g["ba"] = dua.sum(0)
    dfeat = dua @ p["Wa"].T
    # encoder: the max-pool routes each channel's gradient to its argmax point
    for name in ("W2", "b2", "W1", "b1"):
        g[name] = np.zeros_like(p[name])
    for b in range(B):
        e = f["enc"][b]
        arg = e["arg"].copy()
        if arg_override:
            for (bb, c), n in arg_override.items():
                if bb == b:
                    arg[c] = n
        dz2 = np.zeros_like(e["z2"])
        cols = np.arange(dz2.shape[1])
        dz2[arg, cols] = dfeat[b] * (e["z2"][arg, cols] > 0)
        g["W2"] += e["h1"].T @ dz2
        g["b2"] += dz2.sum(0)
        dz1 = (dz2 @ p["W2"].T) * (e["z1"] > 0)
        g["W1"] += xs[b].T @ dz1
        g["b1"] += dz1.sum(0)
    return L / T, g


# ---------------------------------------------------------------------------
# poses <-> y, sampling
# ---------------------------------------------------------------------------
def sixd_to_rot(a) -> np.ndarray:
    """Gram-Schmidt of the two 3-vectors in a[0:3], a[3:6]; R's columns are b1, b2, b1 x b2."""
    a1, a2 = np.asarray(a[0:3], np.float64), np.asarray(a[3:6], np.float64)
    b1 = a1 / max(np.linalg.norm(a1), 1e-8)
    v = a2 - np.dot(b1, a2) * b1
    b2 = v / max(np.linalg.norm(v), 1e-8)
    return np.stack([b1, b2, np.cross(b1, b2)], axis=1)


def pose_to_y(pose12) -> np.ndarray:
    P = np.asarray(pose12, np.float64).reshape(3, 4)
    return np.concatenate([P[:, 0], P[:, 1], P[:, 3] / S_T])


def y_to_pose(y) -> np.ndarray:
    R = sixd_to_rot(y[:6])
    return np.concatenate([R, (np.asarray(y[6:9]) * S_T)[:, None]], axis=1).ravel()


def _u(w) -> float:
    return float(int(w) >> 8) * 2.0 ** -24                 # [0, 1)


def _u_open(w) -> float:
    return float((int(w) >> 8) + 1) * 2.0 ** -24           # (0, 1]


def shoemake_R(u1: float, u2: float, u3: float) -> np.ndarray:
    """Uniform rotation from three uniforms (unit quaternion x, y, z, w)."""
    a, b = math.sqrt(1.0 - u1), math.sqrt(u1)
    x, y = a * math.sin(2 * math.pi * u2), a * math.cos(2 * math.pi * u2)
    z, w = b * math.sin(2 * math.pi * u3), b * math.cos(2 * math.pi * u3)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                     [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                     [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def sample(o: np.ndarray, n: int, seed: int, uniform_frac: float, d_lo: float, d_hi: float,
           philox) -> dict:
    """n poses [n][12] from the mixture row ``o``; ``philox(ctr, key)`` is the
    Philox4x32-10 block function.  Returns the poses, the component of each
    (-1 = uniform fallback) and a flag for draws within 1e-6 of a decision
    boundary (the fallback threshold or a cumulative mixture weight)."""
    lp, mu, ls, _ = mixture(o)
    pi = np.exp(lp)
    cum = np.cumsum(pi)
    key = (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    poses = np.zeros((n, 12))
    comp = np.zeros(n, np.int64)
    flag = np.zeros(n, bool)
    for i in range(n):
        w = np.concatenate([philox((i, j, PHILOX_TAG, 0), key) for j in range(3)])
        uf = _u(w[0])
        flag[i] |= abs(uf - uniform_frac) < 1e-6
        if uf < uniform_frac:
            R = shoemake_R(_u(w[1]), _u(w[2]), _u(w[3]))
            cz, ph = _u(w[4]), 2.0 * math.pi * _u(w[5])
            d = d_lo + (d_hi - d_lo) * _u(w[6])
            sz = math.sqrt(max(0.0, 1.0 - cz * cz))
            t = d * np.array([sz * math.cos(ph), sz * math.sin(ph), cz])
            poses[i] = np.concatenate([R, t[:, None]], axis=1).ravel()
            comp[i] = -1
            continue
        uc = _u(w[1])
        m = int(np.searchsorted(cum, uc, side="right"))
        m = min(m, M - 1)
        flag[i] |= bool(np.any(np.abs(cum[:-1] - uc) < 1e-6))
        z = np.zeros(10)
        for j in range(5):
            r = math.sqrt(-2.0 * math.log(_u_open(w[2 + 2 * j])))
            th = 2.0 * math.pi * _u(w[3 + 2 * j])
            z[2 * j], z[2 * j + 1] = r * math.cos(th), r * math.sin(th)
        y = mu[m] + np.exp(ls[m]) * z[:Y]
        poses[i] = y_to_pose(y)
        comp[i] = m
    return {"poses": poses, "comp": comp, "flag": flag}
