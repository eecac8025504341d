"""GPU parity of the k < F paths against the oracle, through the C ABI
(Sec. 5.3: k contact domains chosen at random per set; Sec. 5.6: fingers
without contact take random joint values and go through the collision
checks), and of realize on sets it cannot realise.

Bars are those of the k = F stages: drawn points bit-exact, links and verdicts
exact outside the oracle's rounding bands, link end points within 1e-5 m.
Stage isolated: each GPU stage gets the oracle's own inputs.
"""
import dataclasses
import math

import numpy as np
import pytest

import oracle
import synth
from tests._realize_bars import check_realize
from tests.test_gpu_parity import _realize_check, _search_check, dev, lgmod, soa

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def _with(w, **kw):
    return dataclasses.replace(w, search=dataclasses.replace(w.search, **kw))


@pytest.mark.parametrize("name,k", [("c3", 3), ("c3", 1), ("c2", 2), ("c1", 2)])
def test_search_k_below_f(name, k):
    w = synth.workload(name, samples=4096 if name != "c1" else None, n_poses=96)
    w = _with(w, k=k)
    ref = oracle.build_field(w.hand, w.field, flags=False)
    Q = oracle.query(w.hand, w.field, ref["bits"], w.obj.pts, w.obj.nrm, w.poses, flags=False)
    spt, sln, ver, acc = _search_check(w, ref["bits"], Q)
    # every drawn contact sits on the finger the oracle chose for it
    fing = oracle.choose_fingers(Q["dom_count"], k, w.search)
    on = sln >= 0
    assert on.sum() > 0
    assert (w.hand.joint_finger[sln[on]] == fing[on]).all()
    assert ((spt >= 0) == (fing >= 0)).all()
    if k == 1:
        assert ver.sum() == 0          # one contact never balances
    else:
        assert len(acc) > 0


@pytest.mark.parametrize("name,k", [("c3", 3), ("c3", 4), ("c1", 2)])
def test_realize_k_below_f(name, k):
    if name == "c3":
        w = synth.workload("c3", samples=8192, n_poses=96)
    else:
        w = synth.workload("c1", with_sdf=True)
    w = _with(w, k=k)
    R, val = _realize_check(w, n_sets_max=2000)
    assert val.sum() > 0 if name == "c3" else True


def test_realize_sets_it_cannot_realise():
    """Invalid links, points, finger order and set ids from the caller give
    not-valid grasps with every finger at its random values, and no read
    through them."""
    lg = lgmod()
    w = _with(synth.workload("c3", samples=8192, n_poses=64), k=3, draws=64)
    k = 3
    ref = oracle.build_field(w.hand, w.field, witness=True, flags=False)
    Q = oracle.query(w.hand, w.field, ref["bits"], w.obj.pts, w.obj.nrm, w.poses, flags=False)
    spt, sln = oracle.draw(w.hand, w.field, ref["bits"], w.obj.pts, w.obj.nrm, w.poses, Q["dom_bits"],
                           Q["dom_count"], w.search)
    V = oracle.verdicts(w.obj.pts, w.obj.nrm, spt, w.search)
    acc = oracle.compact(V["verdict"])[:5]
    assert len(acc) == 5
    S, L = spt.reshape(-1, k).copy(), sln.reshape(-1, k).copy()
    L[acc[0], 1] = -1
    S[acc[1], 0] = w.obj.n
    L[acc[2]] = L[acc[2]][::-1]
    L[acc[3], 2] = w.hand.n_joints          # not a link of the hand
    R = oracle.realize(w.hand, w.field, ref["wit"], w.sdf, w.obj.pts, w.obj.nrm, w.poses, S, L, w.search,
                       acc[:5], w.ik)
    field = lg.lg_field_import(w.hand, w.field, ref["bits"], ref["wit"])
    sdf_vals = dev(w.sdf.values)        # keeps the device copy alive: the struct holds only its address
    sdf = lg.sdf_struct(w.sdf, sdf_vals)
    bad_id = len(w.poses) * w.search.draws
    acc_g = np.append(acc, [bad_id, -1]).astype(np.int32)
    n = len(acc_g)
    bufs = lg.lg_realize(field, sdf, soa(w.obj.pts), soa(w.obj.nrm), dev(w.poses), dev(S.reshape(spt.shape)),
                         dev(L.reshape(spt.shape).astype(np.int8)), k, w.search.draws, dev(acc_g),
                         dev(np.array([n], np.int32)), n, w.ik, sp=w.search)
    torch.cuda.synchronize()
    q = bufs.q.cpu().numpy()
    err = bufs.contact_err.cpu().numpy()
    ang = bufs.contact_ang.cpu().numpy()
    dep = bufs.depth.cpu().numpy()
    val = bufs.valid.cpu().numpy()
    for a in range(4):
        assert np.isinf(err[a]).all() and np.isinf(ang[a]).all() and val[a] == 0
        np.testing.assert_allclose(q[a], R["q"][a], atol=1e-6, rtol=0)   # every finger random
        assert abs(dep[a] - R["depth"][a]) <= 1e-5
    assert np.isfinite(err[4]).all()
    np.testing.assert_allclose(err[4], R["contact_err"][4], atol=1e-5, rtol=0)
    for a in (5, 6):                                   # not set ids
        assert np.isnan(q[a]).all() and np.isinf(err[a]).all() and np.isnan(dep[a]) and val[a] == 0


def test_cone_domains_through_search_and_realize():
    """Cone-query domains hold points where no link of the finger has the
    nearest bin set: those contacts get link -1 and their sets are not
    realisable; the rest follow the oracle."""
    lg = lgmod()
    w = synth.workload("c3", samples=8192, n_poses=48, n_points=4096)
    ref = oracle.build_field(w.hand, w.field, witness=True, flags=False)
    cos_hit = float(np.float32(math.cos(math.radians(15.0))))
    Q = oracle.query_cone(w.hand, w.field, ref["bits"], w.obj.pts, w.obj.nrm, w.poses, cos_hit)
    Q = {"dom_bits": Q["dom_bits"], "dom_count": Q["dom_count"]}
    _search_check(w, ref["bits"], Q)
    # realize on the oracle's own sets (stage isolated)
    k = w.search.k
    spt, sln = oracle.draw(w.hand, w.field, ref["bits"], w.obj.pts, w.obj.nrm, w.poses, Q["dom_bits"],
                           Q["dom_count"], w.search)
    acc = oracle.compact(oracle.verdicts(w.obj.pts, w.obj.nrm, spt, w.search)["verdict"])
    S, L = spt.reshape(-1, k), sln.reshape(-1, k)
    assert (L[acc] < 0).any(), "no accepted set with a contact lacking a link"
    acc = acc[:1500]
    R = oracle.realize(w.hand, w.field, ref["wit"], w.sdf, w.obj.pts, w.obj.nrm, w.poses, S, L, w.search,
                       acc, w.ik)
    field = lg.lg_field_import(w.hand, w.field, ref["bits"], ref["wit"])
    sdf_vals = dev(w.sdf.values)        # keeps the device copy alive: the struct holds only its address
    sdf = lg.sdf_struct(w.sdf, sdf_vals)
    bufs = lg.lg_realize(field, sdf, soa(w.obj.pts), soa(w.obj.nrm), dev(w.poses), dev(spt),
                         dev(sln.astype(np.int8)), k, w.search.draws, dev(acc),
                         dev(np.array([len(acc)], np.int32)), len(acc), w.ik, sp=w.search)
    torch.cuda.synchronize()
    err = bufs.contact_err.cpu().numpy()[:len(acc)]
    val = bufs.valid.cpu().numpy()[:len(acc)]
    no_link = (L[acc] < 0).any(-1)
    assert np.isinf(err[no_link]).all() and (val[no_link] == 0).all()
    assert np.isinf(R["contact_err"][no_link]).all()
    check_realize(w.hand, R, bufs.q.cpu().numpy()[:len(acc)], err, bufs.depth.cpu().numpy()[:len(acc)], val)


def test_pipeline_k_below_f_end_to_end():
    from paper_2511_07418_amd.pipeline import Pipeline
    lg = lgmod()
    w = _with(synth.workload("c3", samples=8192, n_poses=256), k=3)
    field = lg.lg_build_field(w.hand, w.field, keep_witness=True)
    pipe = Pipeline(field, w.obj.pts, w.obj.nrm, w.poses, w.search, sdf=w.sdf, ik=w.ik)
    pipe.step()
    a = pipe.rbuf.q[:pipe.n_acc()].clone()
    va = pipe.rbuf.valid[:pipe.n_acc()].clone()
    pipe.step()
    torch.cuda.synchronize()
    assert pipe.n_acc() > 0
    assert torch.equal(a, pipe.rbuf.q[:pipe.n_acc()]) and torch.equal(va, pipe.rbuf.valid[:pipe.n_acc()])
    assert int(va.sum().item()) > 0
