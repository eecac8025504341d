"""GPU parity of the learned proposer (``lg_prop_*``) against the FP64 oracle
(``oracle/proposer.py``), through the C ABI.

Tolerances.  Every MFMA operand is rounded to bfloat16 (relative error at most
2^-8), products accumulate in FP32.  The oracle's ``bf16=True`` mode rounds the
same operands, so the forward pass differs only by FP32-vs-FP64 accumulation
and by intermediates whose rounding lands on the other side of a bfloat16
rounding boundary: one such flip moves one term of a dot product by at most
2^-8 of its magnitude.  Hence the per-channel bound 2^-7 max_k |h1_k W2_kc| (plus 1e-4 of the sum of
the terms for accumulation order) on pooled features.  The argmax is taken
in the kernel's precision on both sides: it must match wherever the best point
leads the second by more than the accumulation term; elsewhere (dense smooth
objects have many near-ties) the GPU's pick must attain the maximum within
the bound, and the oracle's backward adopts that pick.  The backward products also
round gradients to bfloat16 (the oracle does not), so gradients are compared
at 3e-2 of each tensor's largest entry; a transposed operand or a wrong lane
layout gives O(1) errors.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import proposer as op

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    from paper_2511_07418_amd import lg as _lg
    oracle.build(force=False)
    return _lg


def _objects(n_obj, Np, seed=0):
    xs = []
    for i in range(n_obj):
        o = synth.sphere_object(0.04, Np) if i % 2 == 0 else synth.superquadric_object(seed + i, Np)
        xs.append(np.concatenate([o.pts, o.nrm], axis=1).astype(np.float32))
    return xs


def _enc_bounds(p, e):
    """Per channel, at the oracle's argmax point: (flip, accum) =
    (2^-7 max_k |h1_k W2_kc| + accum, 1e-4 sum_k |h1_k W2_kc|)."""
    terms = np.abs(e["h1"][e["arg"]]) * np.abs(op.bf16_round(p["W2"])).T    # [256][128]
    accum = 1e-4 * terms.sum(1) + 1e-6
    return 2.0 ** -7 * terms.max(1) + accum, accum


def _oracle_inputs(xs):
    return [op.inputs(x[:, :3].astype(np.float64), x[:, 3:].astype(np.float64)) for x in xs]


# 2048 points fill one encoder workgroup; 5000 take three (the last ragged), so
# the pooled keys of several workgroups meet in the 64-bit atomicMax
@pytest.mark.parametrize("B,Np", [(3, 2048), (2, 300), (1, 1), (2, 5000)])
def test_forward_parity(lg, B, Np):
    prop = lg.Proposer(max_batch=4, max_points=max(2048, Np), max_targets=64, seed=11)
    p = op.unflatten(prop.get_params().astype(np.float64))
    xs = _objects(B, Np)
    x = torch.from_numpy(np.stack(xs)).cuda()
    r = prop.forward(x)
    torch.cuda.synchronize()
    feat, arg, out = r["feat"].cpu().numpy(), r["arg"].cpu().numpy(), r["out"].cpu().numpy()
    ox = _oracle_inputs(xs)
    moved = 0
    for b in range(B):
        e = op.encode(p, ox[b], bf16=True)
        flip, accum = _enc_bounds(p, e)
        assert np.all(np.abs(feat[b] - e["feat"]) <= flip), b
        # the GPU's pick attains the maximum within the bound
        z2 = op.bf16_round(e["h1"]) @ op.bf16_round(p["W2"]) + p["b2"]
        picked = np.maximum(z2[arg[b], np.arange(256)], 0.0)
        assert np.all(np.abs(picked - e["feat"]) <= 2.0 * flip)
        # exact argmax wherever the best point leads by more than FP32 accumulation noise;
        # a rounding flip of one intermediate may still move a few (counted)
        # (a channel with a single point has no runner-up: gap = inf, a clear lead)
        lead = np.full_like(e["feat"], np.inf)
        np.multiply(e["gap"], np.abs(e["feat"]), out=lead, where=np.isfinite(e["gap"]))
        clear = (lead > 2.0 * accum) & (e["feat"] > 0.0)
        moved += int((arg[b][clear] != e["arg"][clear]).sum())
        zero = e["feat"] <= 0.0       # every point cut to 0: the tie goes to the lowest index
        np.testing.assert_array_equal(arg[b][zero], 0)
    assert moved <= 0.02 * 256 * B, moved
    # head, isolated: the oracle head (bfloat16 operands) on the GPU's pooled features
    hd = op.head(p, feat.astype(np.float64), bf16=True)
    scale = np.abs(hd["out"]).max()
    assert np.abs(out - hd["out"]).max() <= 1e-2 * scale + 1e-5
    # end to end against the plain FP64 oracle (no operand rounding)
    full = op.forward(p, ox)
    assert np.abs(out - full["out"]).max() <= 5e-2 * np.abs(full["out"]).max()
    prop.release()


def test_forward_repeats_across_batch_sizes(lg):
    """The pooled keys are reset by each pass (no fill kernel): passes of
    3, 1 and 3 objects on one proposer give every object the same bits, and a
    fresh proposer with the same seed agrees."""
    xs = _objects(3, 700, seed=4)
    x3 = torch.from_numpy(np.stack(xs)).cuda()
    x1 = x3[:1].contiguous()
    prop = lg.Proposer(max_batch=4, max_points=700, max_targets=8, seed=21)
    r1 = {k: v.clone() for k, v in prop.forward(x3).items()}
    r2 = {k: v.clone() for k, v in prop.forward(x1).items()}
    r3 = prop.forward(x3)
    fresh = lg.Proposer(max_batch=4, max_points=700, max_targets=8, seed=21)
    r4 = fresh.forward(x3)
    torch.cuda.synchronize()
    for k in ("out", "feat", "arg"):
        assert torch.equal(r1[k], r3[k]) and torch.equal(r1[k], r4[k]), k
        assert torch.equal(r2[k][0], r1[k][0]), k
    prop.release()
    fresh.release()


def test_backward_parity(lg):
    B, Np = 4, 256
    prop = lg.Proposer(max_batch=4, max_points=Np, max_targets=64, seed=5)
    p = op.unflatten(prop.get_params().astype(np.float64))
    xs = _objects(B, Np, seed=3)
    rng = np.random.default_rng(0)
    offsets = np.array([0, 9, 9, 30, 41], np.int32)          # object 1 owns no target
    targets = rng.normal(0, 0.7, size=(int(offsets[-1]), op.Y))
    x = torch.from_numpy(np.stack(xs)).cuda()
    tg = torch.from_numpy(targets.astype(np.float32)).cuda()
    off = torch.from_numpy(offsets).cuda()
    fwd = prop.forward(x)
    loss, grad = prop.backward(x, tg, off)
    torch.cuda.synchronize()
    arg = fwd["arg"].cpu().numpy()
    ox = _oracle_inputs(xs)
    # the oracle takes the GPU's pick where the argmax is a near-tie
    override = {}
    for b in range(B):
        e = op.encode(p, ox[b], bf16=True)
        flip, _ = _enc_bounds(p, e)
        z2 = op.bf16_round(e["h1"]) @ op.bf16_round(p["W2"]) + p["b2"]
        for c in np.nonzero(arg[b] != e["arg"])[0]:
            assert abs(max(z2[arg[b][c], c], 0.0) - e["feat"][c]) <= 2.0 * flip[c]
            override[(b, int(c))] = int(arg[b][c])
    L, g = op.backward(p, ox, targets, offsets, bf16=True, arg_override=override)
    assert float(loss.cpu()[0]) == pytest.approx(L, rel=2e-3)
    gg = op.unflatten(grad.cpu().numpy().astype(np.float64))
    for k, _ in op.LAYERS:
        ref = g[k]
        err = np.abs(gg[k] - ref).max()
        assert err <= 3e-2 * np.abs(ref).max() + 1e-7, (k, err, np.abs(ref).max())
    prop.release()


def test_sampler_parity(lg):
    rng = np.random.default_rng(9)
    o = np.zeros(op.OUT)
    o[:op.M] = rng.normal(0, 1, op.M)
    o[op.M:op.M + op.M * op.Y] = rng.normal(0, 1, op.M * op.Y)
    o[op.M + op.M * op.Y:] = rng.uniform(-3.0, 0.0, op.M * op.Y)
    o32 = o.astype(np.float32)
    n, seed = 3000, 0x1234_5678_9ABC
    poses = lg.lg_prop_sample_mixture(torch.from_numpy(o32).cuda(), n, seed, 0.25, 0.08, 0.12)
    torch.cuda.synchronize()
    g = poses.cpu().numpy().reshape(n, 3, 4)
    ref = op.sample(o32.astype(np.float64), n, seed, 0.25, 0.08, 0.12, oracle.philox)
    r = ref["poses"].reshape(n, 3, 4)
    ok = ~ref["flag"]
    assert ok.mean() > 0.99
    assert np.abs(g[ok][:, :, :3] - r[ok][:, :, :3]).max() <= 1e-4
    assert np.abs(g[ok][:, :, 3] - r[ok][:, :, 3]).max() <= 1e-5
    # edge cases: no poses; all uniform
    assert lg.lg_prop_sample_mixture(torch.from_numpy(o32).cuda(), 0, 1, 0.5).shape == (0, 12)
    pu = lg.lg_prop_sample_mixture(torch.from_numpy(o32).cuda(), 500, 2, 1.0, 0.08, 0.12).cpu().numpy()
    d = np.linalg.norm(pu.reshape(500, 3, 4)[:, :, 3], axis=1)
    assert d.min() >= 0.08 - 1e-6 and d.max() <= 0.12 + 1e-6


def test_training_is_deterministic_and_lowers_the_loss(lg):
    B, Np = 4, 512
    xs = _objects(B, Np, seed=7)
    x = torch.from_numpy(np.stack(xs)).cuda()
    rng = np.random.default_rng(1)
    # targets: two modes per object
    ys = []
    offsets = [0]
    for b in range(B):
        modes = rng.normal(0, 0.8, size=(2, op.Y))
        ys.append(modes[rng.integers(0, 2, 24)] + rng.normal(0, 0.05, size=(24, op.Y)))
        offsets.append(offsets[-1] + 24)
    tg = torch.from_numpy(np.concatenate(ys).astype(np.float32)).cuda()
    off = torch.from_numpy(np.array(offsets, np.int32)).cuda()
    runs = []
    for _ in range(2):
        prop = lg.Proposer(max_batch=B, max_points=Np, max_targets=128, seed=3)
        losses = [float(prop.train_step(x, tg, off, 3e-3).cpu()[0]) for _ in range(60)]
        runs.append((losses, prop.get_params()))
        prop.release()
    assert runs[0][0] == runs[1][0]
    np.testing.assert_array_equal(runs[0][1], runs[1][1])
    losses = runs[0][0]
    assert losses[-1] < losses[0] - 3.0, (losses[0], losses[-1])


def test_proposals_feed_the_unchanged_pipeline(lg):
    from paper_2511_07418_amd.pipeline import Pipeline
    w = synth.workload("c1", n_poses=256)
    field = lg.lg_build_field(w.hand, w.field, keep_witness=False)
    prop = lg.Proposer(max_batch=1, max_points=2048, max_targets=16, seed=1)
    x = torch.from_numpy(np.concatenate([w.obj.pts, w.obj.nrm], axis=1).astype(np.float32)).cuda()[None]
    poses = prop.sample(x, 256, seed=4, uniform_frac=0.5)
    torch.cuda.synchronize()
    P = poses.cpu().numpy().reshape(256, 3, 4)
    np.testing.assert_allclose(np.einsum("nij,nik->njk", P[:, :, :3], P[:, :, :3]),
                               np.broadcast_to(np.eye(3), (256, 3, 3)), atol=1e-5)
    pipe = Pipeline(field, w.obj.pts, w.obj.nrm, P.reshape(256, 12), w.search)
    pipe.query()
    pipe.search()
    torch.cuda.synchronize()
    assert 0 <= pipe.n_acc() <= 256 * w.search.draws
    prop.release()
    field.release()
