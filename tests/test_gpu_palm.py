"""GPU parity of the static-link (palm) contacts (Sec. 5.1) against the
oracle, through the C ABI: palm placements, then the search with each pose's
palm contact as one more fixed contact (verdicts and Alg. 2).

Bars: placements within 2e-5 of the FP64 construction and palm_pt exact
outside the oracle's flags; a pose whose penetration is within 1e-6 of the
margin keeps or rejects the oracle's point, one whose alignment cosine is in
the rotation's branch band matches one of the two branches; unselected poses
untouched; draws bit-exact; verdicts
exact outside |t* - eps| <= 1e-6, t* within 1e-9; Alg. 2 at its own bar.
"""
import dataclasses

import numpy as np
import pytest

import oracle
import synth
from tests.test_gpu_optimize import check_flagged_outcomes
from tests.test_gpu_parity import dev, lgmod, soa

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def _placed(name, n_poses, prob=0.5, seed=9, **kw):
    lg = lgmod()
    w = synth.workload(name, n_poses=n_poses, with_sdf=True, **kw)
    palm = synth.palm_for(name)
    ref = oracle.build_field(w.hand, w.field, flags=False)
    field = lg.lg_field_import(w.hand, w.field, ref["bits"], palm=palm)
    sdf_vals = dev(w.sdf.values)
    sdf = lg.sdf_struct(w.sdf, sdf_vals)
    poses = dev(w.poses)
    pp = lg.lg_place_palm(field, sdf, soa(w.obj.pts), soa(w.obj.nrm), poses, prob, 0.002, seed, request_id=2,
                          pose_offset=5)
    torch.cuda.synchronize()
    O = oracle.place_palm(palm, w.sdf, w.obj.pts, w.obj.nrm, w.poses, prob, 0.002, seed, request_id=2,
                          pose_offset=5)
    return w, palm, ref, field, poses, pp, O, sdf_vals


@pytest.mark.parametrize("name", ["c1", "c3"])
def test_place_palm(name):
    kw = {"samples": 4096} if name == "c3" else {}
    w, palm, ref, field, poses, pp, O, _ = _placed(name, 2048, **kw)
    g_pp = pp.cpu().numpy()
    g_poses = poses.cpu().numpy().astype(np.float64)
    fl = O["pflag"]
    ok = fl == 0
    assert ok.mean() > 0.99
    assert (g_pp[ok] == O["palm_pt"][ok]).all()
    sel = O["sel_pt"] >= 0
    assert ((O["palm_pt"] != -1) == sel).all()
    assert 0.4 < sel.mean() < 0.6
    assert (g_pp[~sel] == -1).all()
    np.testing.assert_array_equal(g_poses[~sel], w.poses[~sel].astype(np.float64))
    rot = (fl & 1) != 0
    err = np.abs(g_poses[sel & ~rot] - O["poses"][sel & ~rot])
    assert err.max() <= 2e-5, err.max()
    # a penetration at the margin: the GPU keeps or rejects the same point
    pen = (fl == 2)
    assert ((g_pp[pen] == O["sel_pt"][pen]) | (g_pp[pen] == -2)).all()
    # a cosine in the rotation's branch band: the pose of one of the two branches,
    # with that branch's outcome
    if rot.any():
        A = oracle.place_palm(palm, w.sdf, w.obj.pts, w.obj.nrm, w.poses, 0.5, 0.002, 9, request_id=2,
                              pose_offset=5, flip=True)
        for g in np.flatnonzero(rot):
            e = [np.abs(g_poses[g] - B["poses"][g]).max() for B in (O, A)]
            assert min(e) <= 2e-5, (g, e)
            B = (O, A)[int(e[1] < e[0])]
            assert g_pp[g] == B["palm_pt"][g] or ((B["pflag"][g] & 2) and g_pp[g] in (B["sel_pt"][g], -2))
    if name == "c3":
        assert (O["palm_pt"] == -2).any()


def test_search_with_palm_contacts():
    lg = lgmod()
    w, palm, ref, field, poses, pp, O, _ = _placed("c3", 128, samples=4096, n_points=8192)
    p32 = O["poses"].astype(np.float32)
    o_pp = O["palm_pt"]
    sp = dataclasses.replace(w.search, k=3, draws=32)
    Q = oracle.query(w.hand, w.field, ref["bits"], w.obj.pts, w.obj.nrm, p32, flags=False)
    bufs = lg.lg_search(field, soa(w.obj.pts), soa(w.obj.nrm), dev(p32), dev(Q["dom_bits"].view(np.int32)),
                        dev(Q["dom_count"].view(np.int32)), sp, palm_pt=dev(o_pp))
    torch.cuda.synchronize()
    spt = bufs.set_pt.cpu().numpy()
    ver = bufs.verdict.cpu().numpy().reshape(-1)
    tst = bufs.tstar.cpu().numpy().reshape(-1)
    acc = bufs.acc_list[:int(bufs.n_acc.item())].cpu().numpy()
    o_spt, _ = oracle.draw(w.hand, w.field, ref["bits"], w.obj.pts, w.obj.nrm, p32, Q["dom_bits"],
                           Q["dom_count"], sp, palm_pt=o_pp)
    assert (spt == o_spt).all()
    assert (spt[o_pp == -2] == -1).all()
    V = oracle.verdicts_palm(w.obj.pts, w.obj.nrm, o_spt, o_pp, sp)
    vf = V["vflag"].astype(bool)
    assert ((ver != V["verdict"]) & ~vf).sum() == 0
    fin = ~np.isnan(V["tstar"])
    assert np.allclose(tst[fin], V["tstar"][fin], atol=1e-9, rtol=0) and np.isnan(tst[~fin]).all()
    assert (acc == np.flatnonzero(ver)).all()
    # the palm contact makes grasps that three fingers alone do not
    V3 = oracle.verdicts(w.obj.pts, w.obj.nrm, o_spt, sp)
    with_palm = np.repeat(o_pp >= 0, sp.draws)
    assert ver[with_palm].mean() > V3["verdict"][with_palm].mean()


def test_optimize_with_palm_contacts():
    lg = lgmod()
    w, palm, ref, field, poses, pp, O, _ = _placed("c3", 48, samples=4096, n_points=4096)
    p32 = O["poses"].astype(np.float32)
    o_pp = O["palm_pt"]
    sp = dataclasses.replace(w.search, k=3, draws=32, opt_outer=1, opt_inner=8, opt_sigma=0.004)
    Q = oracle.query(w.hand, w.field, ref["bits"], w.obj.pts, w.obj.nrm, p32, flags=False)
    bufs = lg.lg_search(field, soa(w.obj.pts), soa(w.obj.nrm), dev(p32), dev(Q["dom_bits"].view(np.int32)),
                        dev(Q["dom_count"].view(np.int32)), sp, palm_pt=dev(o_pp))
    torch.cuda.synchronize()
    spt = bufs.set_pt.cpu().numpy()
    ver = bufs.verdict.cpu().numpy().reshape(-1)
    tst = bufs.tstar.cpu().numpy().reshape(-1)
    d_spt, _ = oracle.draw(w.hand, w.field, ref["bits"], w.obj.pts, w.obj.nrm, p32, Q["dom_bits"],
                           Q["dom_count"], sp, palm_pt=o_pp)
    Opt = oracle.optimize(w.obj.pts, w.obj.nrm, Q["dom_bits"], d_spt, sp, w.hand.n_fingers,
                          dom_count=Q["dom_count"], palm_pt=o_pp)
    k = sp.k
    valid = (d_spt >= 0).all(-1).reshape(-1)
    flag = Opt["oflag"].astype(bool)
    assert flag.sum() <= 0.08 * max(1, valid.sum())
    ok = valid & ~flag
    assert ok.sum() > 0
    same = (spt.reshape(-1, k) == Opt["set_pt"].reshape(-1, k)).all(-1)
    assert same[ok].all()
    assert np.allclose(tst[ok], Opt["tstar"][ok], atol=1e-9, rtol=0)
    assert ((ver != Opt["verdict"]) & ok & ~Opt["vflag"].astype(bool)).sum() == 0
    check_flagged_outcomes(dataclasses.replace(w, poses=p32), sp, Q, d_spt, np.flatnonzero(valid & flag), spt, tst,
                           ver, palm_pt=o_pp)

def test_pipeline_with_palm_contacts():
    from paper_2511_07418_amd.pipeline import Pipeline
    lg = lgmod()
    w = synth.workload("c3", n_poses=512, samples=8192, with_sdf=True)
    palm = synth.palm_for("c3")
    field = lg.lg_build_field(w.hand, w.field, keep_witness=True, palm=palm)
    sdf_vals = dev(w.sdf.values)
    sdf = lg.sdf_struct(w.sdf, sdf_vals)
    poses = dev(w.poses)
    pp = lg.lg_place_palm(field, sdf, soa(w.obj.pts), soa(w.obj.nrm), poses, 0.5, 0.002, 4)
    sp = dataclasses.replace(w.search, k=3)
    pipe = Pipeline(field, w.obj.pts, w.obj.nrm, poses, sp, sdf=w.sdf, ik=w.ik, palm_pt=pp)
    pipe.step()
    a = pipe.valid_sets().clone()
    pipe.step()
    torch.cuda.synchronize()
    assert torch.equal(a, pipe.valid_sets()) and a.numel() > 0
    # valid grasps come from both kinds of poses
    g = (a // sp.draws).long()
    ppc = pp.long()
    assert (ppc[g] >= 0).any() and (ppc[g] == -1).any()
    assert not (ppc[g] == -2).any()


def test_place_palm_needs_a_palm():
    lg = lgmod()
    w = synth.workload("c1", n_poses=4, with_sdf=True)
    field = lg.lg_build_field(w.hand, w.field, keep_witness=False)
    sdf_vals = dev(w.sdf.values)
    sdf = lg.sdf_struct(w.sdf, sdf_vals)
    with pytest.raises(lg.LgError) as ei:
        lg.lg_place_palm(field, sdf, soa(w.obj.pts), soa(w.obj.nrm), dev(w.poses), 0.5, 0.002, 1)
    assert ei.value.status == lg.LG_EINVAL
    with pytest.raises(lg.LgError):
        lg.lg_place_palm(lg.lg_build_field(w.hand, w.field, keep_witness=False, palm=synth.palm_for("c1")), sdf,
                         soa(w.obj.pts), soa(w.obj.nrm), dev(w.poses), 1.5, 0.002, 1)
