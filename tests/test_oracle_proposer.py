"""Pins of the proposer oracle (``oracle/proposer.py``) against things other
than itself:

* the mixture NLL against scipy's normal log-density and logsumexp;
* the hand-written backward against torch autograd in float64 (an
  independent derivative mechanism) and the output gradient against central
  differences;
* bfloat16 rounding against torch's float32 -> bfloat16 conversion;
* the 6-D rotation map against its closed-form properties;
* PointNet permutation invariance;
* the sampler against the mixture's moments and weights and the uniform
  fallback against Haar-measure moments.
"""
import math

import numpy as np
import pytest
from scipy.special import logsumexp
from scipy.stats import chi2, norm

import oracle
from oracle import proposer as op

torch = pytest.importorskip("torch")


def _rand_params(rng, dims=None, scale=0.3):
    dims = dims or {"H1": op.H1, "H2": op.H2, "HH": op.HH}
    shapes = {"W1": (op.D_IN, dims["H1"]), "b1": (dims["H1"],), "W2": (dims["H1"], dims["H2"]),
              "b2": (dims["H2"],), "Wa": (dims["H2"], dims["HH"]), "ba": (dims["HH"],),
              "Wb": (dims["HH"], dims["HH"]), "bb": (dims["HH"],), "Wc": (dims["HH"], op.OUT),
              "bc": (op.OUT,)}
    p = {k: rng.normal(0, scale, size=s) for k, s in shapes.items()}
    return p


def _rand_out(rng):
    o = rng.normal(0, 1, size=op.OUT)
    o[op.M + op.M * op.Y:] = rng.uniform(-1.5, 0.5, size=op.M * op.Y)   # inside the clamp
    return o


def test_nll_matches_scipy():
    rng = np.random.default_rng(1)
    for _ in range(20):
        o = _rand_out(rng)
        y = rng.normal(0, 1, size=op.Y)
        logits = o[:op.M]
        mu = o[op.M:op.M + op.M * op.Y].reshape(op.M, op.Y)
        sig = np.exp(o[op.M + op.M * op.Y:].reshape(op.M, op.Y))
        lpi = logits - logsumexp(logits)
        ref = -logsumexp(lpi + norm.logpdf(y[None, :], mu, sig).sum(axis=1))
        assert op.nll(o, y) == pytest.approx(ref, rel=1e-12, abs=1e-12)


def test_log_sigma_clamp():
    o = np.zeros(op.OUT)
    o[op.M + op.M * op.Y:] = -50.0
    _, _, ls, inside = op.mixture(o)
    assert np.all(ls == op.LS_MIN) and not inside.any()


def test_grad_out_central_differences():
    rng = np.random.default_rng(2)
    o = _rand_out(rng)
    ys = rng.normal(0, 1, size=(5, op.Y))
    g = op.grad_out(o, ys, 1.0)
    f = lambda oo: sum(op.nll(oo, y) for y in ys)
    h = 1e-6
    for j in range(op.OUT):
        e = np.zeros(op.OUT)
        e[j] = h
        fd = (f(o + e) - f(o - e)) / (2 * h)
        assert g[j] == pytest.approx(fd, rel=1e-5, abs=1e-6), j


def _torch_loss(p, xs, targets, offsets):
    """The same network and loss built from torch primitives (float64)."""
    T = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in p.items()}
    feats = []
    for x in xs:
        xt = torch.tensor(x, dtype=torch.float64)
        h1 = torch.relu(torch.nn.functional.linear(xt, T["W1"].t(), T["b1"]))
        h2 = torch.relu(torch.nn.functional.linear(h1, T["W2"].t(), T["b2"]))
        feats.append(h2.max(dim=0).values)
    f = torch.stack(feats)
    ua = torch.relu(f @ T["Wa"] + T["ba"])
    ub = torch.relu(ua @ T["Wb"] + T["bb"])
    o = ub @ T["Wc"] + T["bc"]
    M, Y = op.M, op.Y
    tot = 0.0
    for b in range(len(xs)):
        lpi = torch.log_softmax(o[b, :M], dim=0)
        mu = o[b, M:M + M * Y].reshape(M, Y)
        ls = torch.clamp(o[b, M + M * Y:].reshape(M, Y), op.LS_MIN, op.LS_MAX)
        for t in range(int(offsets[b]), int(offsets[b + 1])):
            y = torch.tensor(targets[t], dtype=torch.float64)
            dist = torch.distributions.Normal(mu, torch.exp(ls))
            tot = tot - torch.logsumexp(lpi + dist.log_prob(y).sum(dim=1), dim=0)
    L = tot / int(offsets[-1])
    L.backward()
    return float(L.detach()), {k: v.grad.numpy() for k, v in T.items()}


@pytest.mark.parametrize("dims", [{"H1": 5, "H2": 7, "HH": 6}, {"H1": op.H1, "H2": op.H2, "HH": op.HH}])
def test_backward_matches_torch_autograd(dims):
    rng = np.random.default_rng(3)
    p = _rand_params(rng, dims)
    xs = [rng.normal(0, 1, size=(n, op.D_IN)) for n in (9, 13, 1)]
    offsets = np.array([0, 3, 3, 7])          # object 1 has no targets
    targets = rng.normal(0, 1, size=(7, op.Y))
    L, g = op.backward(p, xs, targets, offsets)
    Lt, gt = _torch_loss(p, xs, targets, offsets)
    assert L == pytest.approx(Lt, rel=1e-12)
    for k in p:
        np.testing.assert_allclose(g[k], gt[k], rtol=1e-9, atol=1e-12, err_msg=k)


def test_bf16_round_matches_torch():
    rng = np.random.default_rng(4)
    a = np.concatenate([rng.normal(0, 1, 10000) * 10.0 ** rng.integers(-8, 8, 10000),
                        np.array([0.0, -0.0, 1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 65504.0])]).astype(np.float32)
    ref = torch.tensor(a).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(op.bf16_round(a), ref)


def test_sixd_rotation_properties():
    rng = np.random.default_rng(5)
    for _ in range(200):
        a = rng.normal(0, 1, size=6)
        R = op.sixd_to_rot(a)
        np.testing.assert_allclose(R.T @ R, np.eye(3), atol=1e-12)
        assert np.linalg.det(R) == pytest.approx(1.0, abs=1e-12)
        # b1 is a1's direction; b2 lies in span(a1, a2) on a2's side
        np.testing.assert_allclose(R[:, 0], a[:3] / np.linalg.norm(a[:3]), atol=1e-12)
        assert np.dot(R[:, 1], a[3:]) > 0 and abs(np.dot(np.cross(a[:3], a[3:]), R[:, 1])) < 1e-9
    # the two columns of a rotation map back to it exactly
    from scipy.spatial.transform import Rotation
    for R in Rotation.random(50, random_state=6).as_matrix():
        pose = np.concatenate([R, np.array([[0.01], [0.02], [0.09]])], axis=1).ravel()
        np.testing.assert_allclose(op.y_to_pose(op.pose_to_y(pose)), pose, atol=1e-12)


def test_pointnet_permutation_invariance():
    rng = np.random.default_rng(7)
    p = _rand_params(rng)
    x = rng.normal(0, 1, size=(300, op.D_IN))
    perm = rng.permutation(300)
    e1, e2 = op.encode(p, x), op.encode(p, x[perm])
    np.testing.assert_allclose(e1["feat"], e2["feat"], rtol=1e-14, atol=0)
    pos = e1["feat"] > 0          # a channel cut to 0 at every point ties; its argmax is the first index
    assert pos.sum() > 100
    np.testing.assert_array_equal(perm[e2["arg"]][pos], e1["arg"][pos])


def test_sampler_matches_mixture_moments():
    oracle.build(force=False)
    rng = np.random.default_rng(8)
    o = np.zeros(op.OUT)
    o[:op.M] = np.log(np.array([1, 2, 3, 4, 1, 2, 3, 4], float))
    mu = rng.normal(0, 1, size=(op.M, op.Y))
    ls = rng.uniform(-2.0, -0.5, size=(op.M, op.Y))
    o[op.M:op.M + op.M * op.Y] = mu.ravel()
    o[op.M + op.M * op.Y:] = ls.ravel()
    n = 12000
    s = op.sample(o, n, seed=123, uniform_frac=0.2, d_lo=0.08, d_hi=0.12, philox=oracle.philox)
    comp = s["comp"]
    # fallback frequency
    nu = int((comp == -1).sum())
    assert abs(nu - 0.2 * n) < 4 * math.sqrt(n * 0.2 * 0.8)
    # component frequencies: chi-square against the softmax weights
    pi = np.array([1, 2, 3, 4, 1, 2, 3, 4], float) / 20.0
    cnt = np.bincount(comp[comp >= 0], minlength=op.M)
    exp = pi * cnt.sum()
    assert ((cnt - exp) ** 2 / exp).sum() < chi2.ppf(0.999, op.M - 1)
    # translations: mean and std of t / S_T per component
    for m in range(op.M):
        t = s["poses"][comp == m][:, [3, 7, 11]] / op.S_T
        sd = np.exp(ls[m, 6:9])
        se = sd / math.sqrt(len(t))
        assert np.all(np.abs(t.mean(0) - mu[m, 6:9]) < 5 * se)
        assert np.all(np.abs(t.std(0) / sd - 1.0) < 5 / math.sqrt(2 * len(t)))
    # rotations are proper; the uniform branch has Haar moments E[R] = 0
    Rs = s["poses"].reshape(n, 3, 4)[:, :, :3]
    np.testing.assert_allclose(np.einsum("nij,nik->njk", Rs, Rs), np.broadcast_to(np.eye(3), (n, 3, 3)),
                               atol=1e-9)
    Ru = Rs[comp == -1]
    assert np.all(np.abs(Ru.mean(0)) < 5 * math.sqrt(1.0 / 3.0 / len(Ru)))
    tu = s["poses"][comp == -1][:, [3, 7, 11]]
    d = np.linalg.norm(tu, axis=1)
    assert d.min() >= 0.08 - 1e-12 and d.max() <= 0.12 + 1e-12 and tu[:, 2].min() >= 0.0
